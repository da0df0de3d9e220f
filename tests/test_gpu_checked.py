"""The checked build of the library (libgsff_checked.so) on the GPU.

The checked build tests every index its kernels take from data (a sort
destination, a Gaussian id at a depth rank or in a tile list, a tile range, a
walked-list entry, an adjoint work item, row or slot) against what it
addresses; a failed test skips the access and is recorded in the workspace's
status word (GSFF_FLAG_CHECK, gsff_read_checks).  Here:

* on the scenes of the parity suite -- both binning paths, both adjoint
  reduction modes, the explicit and the fused-L1 upstream, several channel
  passes, a BF16 payload, a pair-capacity overflow -- and at full size (the
  benchmark's 200k-Gaussian frame, the adjoint's atomic fallback, 1M
  Gaussians at 1200x680 with a BF16 payload) no test fails, and the outputs
  and gradients are those of the release build;
* conditions forced from the host are reported at their site, with every
  access still inside the workspace: a super-tile range that ends past the
  frame's pairs (the extra entries hold a valid id and an empty tile mask),
  and a walked-list entry set to an id past P before the adjoint.
"""
import numpy as np
import pytest

import helpers as H
from paper_2504_19409_amd import scenegen as sg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_19409_amd import _capi
    _capi.load()
    with _capi.checked_library():  # raises if the checked build is missing
        pass


def _capi():
    from paper_2504_19409_amd import _capi as c
    return c


def _scene(kind, C):
    if kind == "tiny":
        sc, _ = sg.workload_scene("tiny")
        if C != sc.C:
            sc.feat = np.random.default_rng(101).normal(size=(sc.P, C)).astype(np.float32)
        return sc
    if kind == "ragged":
        return sg.make_scene(3000, 70, 50, 50.0, 50.0, 35.0, 25.0, C, seed=11)
    if kind == "rotated":
        rng = np.random.default_rng(12)
        vm, _ = sg.perturbed_viewmat(rng, sg.identity_viewmat(), 0.1, 10.0)
        return sg.make_scene(4000, 96, 64, 70.0, 70.0, 48.0, 32.0, C, seed=12, viewmat=vm)
    if kind == "dense":
        sc = sg.make_scene(6000, 64, 64, 60.0, 60.0, 32.0, 32.0, C, seed=13)
        sc.log_scales += 0.7
        return sc
    raise ValueError(kind)


def _render(sc, settings, l1, feat_dtype=None, max_pairs=None):
    """Forward and adjoint of one frame with the library currently selected;
    returns the outputs, the gradients, the status flags and the check record."""
    fr, _ = H.make_frame(sc, torch, settings=settings, max_pairs=max_pairs,
                         feat_dtype=feat_dtype)
    outs = fr.forward()
    flags, npairs = fr.read_status()
    res = {"flags": flags, "npairs": npairs}
    if flags & _capi().FLAG_PAIR_OVERFLOW:
        res["checks"] = fr.read_checks()
        return res
    W, Hh, C = sc.camera.width, sc.camera.height, sc.C
    grads = fr.make_grads()
    rng = np.random.default_rng(sc.P + 3)
    if l1:
        t_rgb, t_depth, t_feat = sg.make_targets(rng, W, Hh, C)
        targets = [torch.from_numpy(t).cuda() for t in (t_rgb, t_depth)] + [None]
        targets.append(torch.from_numpy(t_feat).cuda() if C else None)
        fr.backward_l1(outs, targets, (1.0, 0.5, 0.0, 1.0), grads)
    else:
        ups = sg.upstream_signs(rng, W, Hh, C)
        dev = [torch.from_numpy(a).cuda() if a is not None else None for a in ups]
        fr.backward(*dev, grads)
    res["checks"] = fr.read_checks()
    res["flags"] = fr.read_status()[0]
    res.update({k: o.float().cpu().numpy() for k, o in zip(("rgb", "depth", "alpha", "feat"), outs)})
    res["grads"] = {k: v.cpu().numpy() for k, v in grads.items()}
    return res


CASES = [
    ("tiny", 16, {}, False, None),
    ("ragged", 5, {}, True, None),
    ("rotated", 16, {"bin_mode": 1}, False, None),
    ("dense", 16, {"deterministic": 1}, True, None),
    ("ragged", 80, {}, False, None),         # two channel passes
    ("rotated", 32, {}, True, torch.bfloat16),
]


@pytest.mark.parametrize("kind,C,kw,l1,fdt", CASES,
                         ids=["tiny", "ragged-l1", "rotated-keysort", "dense-det-l1",
                              "ragged-c80", "rotated-bf16-l1"])
def test_checked_build_clean_and_equal_to_release(kind, C, kw, l1, fdt):
    sc = _scene(kind, C)
    st = _capi().default_settings(**kw)
    rel = _render(sc, st, l1, fdt)
    with _capi().checked_library():
        chk = _render(sc, st, l1, fdt)
    assert chk["checks"]["failures"] == 0, chk["checks"]
    assert chk["flags"] == 0 and rel["flags"] == 0, (chk["flags"], rel["flags"])
    assert rel["checks"]["failures"] == 0  # the release build tests nothing
    diffs = {}
    for k in ("rgb", "depth", "alpha", "feat"):
        a, b = chk[k], rel[k]
        diffs[k] = float(np.abs(a - b).max()) if a.size else 0.0
        assert np.allclose(a, b, rtol=1e-6, atol=1e-6), (k, diffs[k])
    for k, g in rel["grads"].items():
        diffs["d_" + k] = H.rel_l2(chk["grads"][k], g)
        # the default reduction adds with float atomics, in no fixed order
        # (run-to-run spread below 2.5e-4); the fixed-order mode is exact
        tol = 5e-4 if not kw.get("deterministic") else 1e-6
        assert diffs["d_" + k] <= tol, (k, diffs["d_" + k])
    print(f"checked vs release [{kind} C={C} {kw} l1={l1}]: " +
          ", ".join(f"{k} {v:.1e}" for k, v in diffs.items()), flush=True)


def test_checked_build_pair_overflow_is_not_a_failed_check():
    sc = _scene("ragged", 5)
    with _capi().checked_library():
        res = _render(sc, _capi().default_settings(), False, max_pairs=1000)
    assert res["flags"] & _capi().FLAG_PAIR_OVERFLOW
    assert not res["flags"] & _capi().FLAG_CHECK
    assert res["checks"]["failures"] == 0


def _staged_frame(sc):
    fr, _ = H.make_frame(sc, torch)
    for stage in ("gsff_preprocess", "gsff_sort_depth", "gsff_bin", "gsff_sort_tiles",
                  "gsff_tile_ranges"):
        fr.call_stage(stage)
    return fr


def test_forced_tile_range_past_the_pairs_is_reported():
    sc = _scene("ragged", 5)
    c = _capi()
    with c.checked_library():
        fr = _staged_frame(sc)
        torch.cuda.synchronize()
        ref = [o.clone() for o in fr.forward()]
        fr = _staged_frame(sc)
        torch.cuda.synchronize()
        lay = fr.layout
        nsuper = lay.super_x * lay.super_y
        rng_v = fr.ws_view("tile_ranges", torch.int32, 2 * nsuper).view(nsuper, 2)
        status = fr.ws_view("status", torch.int32, 8)
        pairs = int(status[2].item())
        r = rng_v.cpu().numpy()
        s = int(np.nonzero(r[:, 1] > r[:, 0])[0].max())  # the last non-empty super-tile
        assert r[s, 1] == pairs
        end = min(pairs + 37, fr.max_pairs)
        assert end > pairs
        # the entries past the frame's pairs: Gaussian 0, no tile of the super-tile
        fr.ws_view("pair_keys", torch.int32, end)[pairs:end] = 0
        fr.ws_view("pair_masks", torch.int16, end)[pairs:end] = 0
        rng_v[s, 1] = end
        outs = fr.alloc_outputs()
        fr.composite_fwd(outs)
        chk = fr.read_checks()
        flags = fr.read_status()[0]
    assert flags & c.FLAG_CHECK
    sx, sy = s % lay.super_x, s // lay.super_x
    ntile = (min(4, lay.tiles_x - 4 * sx)) * (min(4, lay.tiles_y - 4 * sy))
    assert chk == {"failures": ntile, "site": "tile_range", "index": end, "limit": pairs + 1}, chk
    # nothing past the pairs was accepted: the images are those of the intact frame
    for a, b in zip(outs, ref):
        assert torch.equal(a, b)


def test_forced_walked_id_past_p_is_reported_by_the_adjoint():
    sc = _scene("ragged", 5)
    c = _capi()
    P = sc.P
    with c.checked_library():
        fr, _ = H.make_frame(sc, torch)
        outs = fr.forward()
        lay = fr.layout
        ntiles = lay.tiles_x * lay.tiles_y
        cr = fr.ws_view("tile_list_ranges", torch.int32, 2 * ntiles).view(ntiles, 2).cpu().numpy()
        t = int(np.argmax(cr[:, 1] - cr[:, 0]))  # the longest walk
        pos = int(cr[t, 0]) + 3
        assert cr[t, 1] - cr[t, 0] > 3
        lists = fr.ws_view("tile_lists", torch.int32, pos + 1)
        lists[pos] = P + 7
        assert fr.read_checks()["failures"] == 0  # the forward itself was clean
        rng = np.random.default_rng(5)
        ups = sg.upstream_signs(rng, sc.camera.width, sc.camera.height, sc.C)
        dev = [torch.from_numpy(a).cuda() if a is not None else None for a in ups]
        grads = fr.make_grads()
        fr.backward(*dev, grads)
        chk = fr.read_checks()
        flags = fr.read_status()[0]
    assert flags & c.FLAG_CHECK
    assert chk == {"failures": 1, "site": "list_id", "index": P + 7, "limit": P}, chk
    for v in grads.values():
        assert torch.isfinite(v).all()


def _sized_frame(sc, feat_dtype=None):
    fr, _ = H.make_frame(sc, torch, feat_dtype=feat_dtype)
    fr.forward()
    n = fr.read_status()[1]
    fr, _ = H.make_frame(sc, torch, feat_dtype=feat_dtype, max_pairs=int(n * 1.05) + 4096)
    return fr


def _l1_run(sc, feat_dtype=None):
    """Forward and fused-L1 adjoint (dense seeded targets, the benchmark's loss
    weights) on a frame sized from a first forward; images, loss, flags and
    the check record."""
    fr = _sized_frame(sc, feat_dtype)
    outs = fr.forward()
    W, Hh, C = sc.camera.width, sc.camera.height, sc.C
    t_rgb, t_depth, t_feat = sg.make_targets(np.random.default_rng(31), W, Hh, C)
    targets = [torch.from_numpy(t).cuda() for t in (t_rgb, t_depth)] + [None]
    targets.append(torch.from_numpy(t_feat).cuda() if C else None)
    grads = fr.make_grads()
    loss = torch.zeros(1, device="cuda")
    fr.backward_l1(outs, targets, (1.0, 1.0, 0.0, 1.0), grads, loss)
    return dict(outs=[o.clone() for o in outs], loss=float(loss.item()),
                flags=fr.read_status()[0], checks=fr.read_checks(),
                grads={k: v.cpu().numpy() for k, v in grads.items()})


@pytest.mark.parametrize("case", ["frame", "rows-overflow", "mixed-1M"])
def test_checked_build_at_full_size(case):
    """The benchmark's frame (200k Gaussians, 640x480, 16 FP32 channels, the
    fused-L1 adjoint with dense targets), a frame whose walked pairs overflow
    the adjoint's partial rows (the atomic fallback) and the 1M-Gaussian
    1200x680 frame with a 64-channel BF16 payload: the checked build records
    no failure and renders the release build's images bit for bit."""
    fdt = None
    if case == "frame":
        sc, _ = sg.workload_scene("frame")
    elif case == "rows-overflow":
        sc = sg.make_scene(300, 320, 240, 260.0, 260.0, 160.0, 120.0, 8, seed=41)
        sc.log_scales += 1.8
        sc.logit_opacity = np.full_like(sc.logit_opacity, -3.0)
    else:
        cfg = dict(sg.WORKLOADS["mixed"])
        seed = cfg.pop("seed")
        sc = sg.make_scene(rng=np.random.default_rng(seed), seed=seed, **cfg)
        fdt = torch.bfloat16
    rel = _l1_run(sc, fdt)
    with _capi().checked_library():
        chk = _l1_run(sc, fdt)
    assert chk["checks"]["failures"] == 0, chk["checks"]
    assert chk["flags"] == 0 and rel["flags"] == 0
    for a, b in zip(chk["outs"], rel["outs"]):
        assert torch.equal(a, b)
    assert chk["loss"] == pytest.approx(rel["loss"], rel=1e-5)
    errs = {k: H.rel_l2(chk["grads"][k], g) for k, g in rel["grads"].items()}
    assert max(errs.values()) <= 5e-4, errs  # order of float atomics only
    print(f"checked vs release [{case}]: " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()),
          flush=True)
