"""Full-size workloads the oracle cannot render whole in seconds, checked on
what it can compute exactly at that size:

* forward outputs at sampled pixels (the oracle renders just those pixels);
* every gradient group for an upstream that is non-zero only at sampled
  pixels (the oracle skips pixels with zero upstream, which changes nothing).

Workloads: 1M Gaussians at 1200x680 with 64 BF16 feature channels (the mixed-
precision case), and the 8-view keyframe window (1M Gaussians, 32 BF16
channels, views alternating 640x480 and 1200x680).
"""
import time

import numpy as np
import pytest

import helpers as H
from paper_2504_19409_amd import scenegen as sg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GRADS = ["means", "log_scales", "quats", "logit_opacity", "rgb", "feat", "pose"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_19409_amd import _capi
    _capi.load()


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


def _sparse_upstream(rng, W, Hh, C, n):
    HW = W * Hh
    idx = rng.choice(HW, n, replace=False)
    py, px = np.divmod(idx, W)
    g = [np.zeros((3, Hh, W), np.float32), np.zeros((Hh, W), np.float32),
         np.zeros((Hh, W), np.float32), np.zeros((C, Hh, W), np.float32)]
    sgn = lambda *s: (rng.integers(0, 2, size=s) * 2 - 1).astype(np.float32)
    g[0][:, py, px] = sgn(3, n) / n
    g[1][py, px] = sgn(n) / n
    g[2][py, px] = sgn(n) / n
    g[3][:, py, px] = sgn(C, n) / n
    return g, px, py


def test_mixed_precision_full_size(orc):
    """1M Gaussians, 1200x680, 64-channel BF16 payload, FP32 compositing."""
    cfg = dict(sg.WORKLOADS["mixed"])
    seed = cfg.pop("seed")
    rng = np.random.default_rng(seed)
    sc = sg.make_scene(rng=rng, seed=seed, **cfg)
    fr, _ = H.make_frame(sc, torch, feat_dtype=torch.bfloat16)
    fr.forward()
    flags, n = fr.read_status()
    fr, _ = H.make_frame(sc, torch, feat_dtype=torch.bfloat16, max_pairs=int(n * 1.05) + 4096)
    outs = fr.forward()
    W, Hh, C = sc.camera.width, sc.camera.height, sc.C
    ups, px, py = _sparse_upstream(rng, W, Hh, C, 3000)
    grads = fr.make_grads()
    fr.backward(*[torch.from_numpy(u).cuda() for u in ups], grads)
    torch.cuda.synchronize()
    assert fr.read_status()[0] == 0
    rounded = sg.bf16_to_f32(sg.round_bf16(sc.feat)).astype(np.float64)
    p, c = orc.scene_dicts(sc)
    p_r = dict(p, feat=rounded)
    o = orc.render_pixels(p_r, c, px, py)
    g = {k: v.cpu().numpy() for k, v in zip(["rgb", "depth", "alpha", "feat"], outs)}
    errs = dict(rgb=H.rel_l2(g["rgb"][:, py, px].T, o["rgb"]),
                depth=H.rel_l2(g["depth"][py, px], o["depth"]),
                alpha=H.rel_l2(g["alpha"][py, px], o["alpha"]),
                feat=H.rel_l2(g["feat"][:, py, px].T, o["feat"]))
    print("errors[mixed 1M 1200x680 BF16x64, 3000 pixels] forward relL2 (vs the BF16-rounded "
          "features): " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
    for k, v in errs.items():
        assert v <= H.TOL_FWD, (k, v)
    # error against the unrounded FP32 features, per 16-channel group
    o32 = orc.render_pixels(p, c, px, py)
    for g0 in range(0, 64, 16):
        e = H.rel_l2(g["feat"][g0:g0 + 16, py, px].T, o32["feat"][:, g0:g0 + 16])
        print(f"errors[mixed 1M 1200x680 BF16x64, 3000 pixels] channels {g0}-{g0 + 15}: "
              f"relL2 vs the FP32 features {e:.2e}", flush=True)
        assert e <= H.TOL_BF16
    ob = orc.backward(p_r, c, dict(g_rgb=ups[0], g_depth=ups[1], g_alpha=ups[2], g_feat=ups[3]))
    amb = orc.ambiguous(p_r, c, H.MARGIN, px=px, py=py)
    rep = {}
    H.check_grads({k: v.cpu().numpy() for k, v in grads.items()}, ob, GRADS, flags=amb,
                  report=rep)
    print("errors[mixed 1M 1200x680 BF16x64, 3000 pixels] gradient relL2: " +
          ", ".join(f"{k} {v['rel_l2']:.2e}" for k, v in rep.items()), flush=True)


def test_keyframe_window_full_size(orc):
    """8 views of 1M Gaussians (32 BF16 channels), alternating 640x480 and
    1200x680 on a 2 m arc, one graph: accumulated gradients equal the per-view
    sum, and one view's gradients match the oracle for a sparse upstream."""
    from paper_2504_19409_amd.rasterizer import CameraSpec
    from paper_2504_19409_amd.window import KeyframeWindow
    rng = np.random.default_rng(5)
    P, C = 1_000_000, 32
    sc = sg.make_scene(P, 640, 480, 525.0, 525.0, 320.0, 240.0, C, seed=5, rng=rng)
    vms = sg.arc_viewmats(rng, 8, radius=3.0, arc=2.0, jitter_deg=2.0)
    sizes = [(640, 480, 525.0), (1200, 680, 600.0)] * 4
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    geom = dict(means=t(sc.means), log_scales=t(sc.log_scales), quats=t(sc.quats),
                logit_opacity=t(sc.logit_opacity), rgb=t(sc.rgb))
    feat = t(sc.feat).to(torch.bfloat16)
    views = [(t(vm), CameraSpec(W, Hh, f, f, W / 2, Hh / 2)) for (W, Hh, f), vm in zip(sizes, vms)]
    # targets: each view's own render, perturbed at sampled pixels only, so the
    # L1 upstream sign(out - target) is non-zero exactly there
    targets = []
    for (vm, cam) in views:
        tg = [torch.zeros((3, cam.height, cam.width), device="cuda"),
              torch.zeros((cam.height, cam.width), device="cuda"), None,
              torch.zeros((C, cam.height, cam.width), device="cuda")]
        targets.append(tg)
    win = KeyframeWindow(geom, feat, views, targets, weights=(1.0, 1.0, 0.0, 1.0))
    for v, fr in enumerate(win.frames):
        outs = fr.forward(outs=win.outs[v])
        win.targets[v][0].copy_(outs[0])
        win.targets[v][1].copy_(outs[1])
        win.targets[v][3].copy_(outs[3].float())
    picks = []
    for v, (vm, cam) in enumerate(views):
        idx = rng.choice(cam.width * cam.height, 2000, replace=False)
        py, px = np.divmod(idx, cam.width)
        picks.append((px, py))
        tpx, tpy = torch.from_numpy(px).cuda(), torch.from_numpy(py).cuda()
        win.targets[v][0][:, tpy, tpx] += 0.25
        win.targets[v][1][tpy, tpx] += 0.25
        win.targets[v][3][:, tpy, tpx] += 0.25
    win.capture()
    win.replay()
    torch.cuda.synchronize()
    n = 5
    t0 = time.perf_counter()
    for _ in range(n):
        win.replay()
    torch.cuda.synchronize()
    print(f"\nwindow step (8 views, fwd + bwd, graph replay): {(time.perf_counter() - t0) / n * 1e3:.2f} ms")
    acc = {k: v.clone() for k, v in win.grads.items()}
    # property at any size: the window's accumulation equals the sum of views
    summed = {k: torch.zeros_like(v) for k, v in acc.items()}
    for v, fr in enumerate(win.frames):
        fr.forward(outs=win.outs[v])
        g = {k: torch.empty_like(x) for k, x in acc.items()}
        g["pose"] = torch.empty(6, device="cuda")
        fr.backward_l1(win.outs[v], win.targets[v], win.weights, g)
        for k in acc:
            summed[k] += g[k]
        assert H.rel_l2(g["pose"].cpu().numpy(), win.pose[v].cpu().numpy()) <= 1e-5
    torch.cuda.synchronize()
    for k in acc:
        assert H.rel_l2(acc[k].cpu().numpy(), summed[k].cpu().numpy()) <= 1e-5, k
    # oracle: the last (1200x680) view with its sparse upstream
    v = 7
    fr = win.frames[v]
    outs = fr.forward(outs=win.outs[v])
    g = {k: torch.empty_like(x) for k, x in acc.items()}
    g["pose"] = torch.empty(6, device="cuda")
    fr.backward_l1(outs, win.targets[v], win.weights, g)
    torch.cuda.synchronize()
    (W, Hh, f), vm = sizes[v], vms[v]
    # the upstream the targets define: out - target = -0.25 at the picked
    # pixels of every group in the loss, exactly zero elsewhere
    px, py = picks[v]
    ups = [np.zeros((3, Hh, W)), np.zeros((Hh, W)), np.zeros((Hh, W)), np.zeros((C, Hh, W))]
    ups[0][:, py, px] = -1.0 / ups[0].size
    ups[1][py, px] = -1.0 / ups[1].size
    ups[3][:, py, px] = -1.0 / ups[3].size
    rounded = sg.bf16_to_f32(sg.round_bf16(sc.feat)).astype(np.float64)
    p, _ = orc.scene_dicts(sc)
    p = dict(p, feat=rounded)
    cam = dict(width=W, height=Hh, fx=f, fy=f, cx=W / 2, cy=Hh / 2, viewmat=vm)
    ob = orc.backward(p, cam, dict(g_rgb=ups[0], g_depth=ups[1], g_alpha=ups[2], g_feat=ups[3]))
    amb = orc.ambiguous(p, cam, H.MARGIN, px=px, py=py)
    rep = {}
    H.check_grads({k: x.cpu().numpy() for k, x in g.items()}, ob, GRADS, flags=amb, report=rep)
    print(f"errors[window view {v} 1200x680 BF16x32, 2000 pixels] gradient relL2: " +
          ", ".join(f"{k} {x['rel_l2']:.2e}" for k, x in rep.items()), flush=True)


@pytest.mark.parametrize("W,Hh,f", [(1920, 1088, 1000.0), (3840, 2160, 2000.0)])
def test_large_frame_fused_l1(orc, W, Hh, f):
    """50k Gaussians, 16 FP32 channels on large frames: 1920x1088 has 8160
    tiles (more than the 2048 whose ranges the fused L1 pass's item workgroup
    holds in registers), 510 super-tiles (the binning's range scan runs in two
    chunks) and 196 slot blocks; 3840x2160 has 32400 tiles (more than the 8192
    of the explicit path's 1024-thread item kernel) and 2040 super-tiles.
    The forward on sampled pixels against the oracle; the fused-L1 adjoint
    against the oracle for targets 0.25 above the render at sampled pixels,
    so the upstream is -1/numel there and zero elsewhere; and the explicit
    adjoint given that same upstream."""
    rng = np.random.default_rng(81)
    C = 16
    sc = sg.make_scene(50_000, W, Hh, f, f, W / 2, Hh / 2, C, seed=81, rng=rng)
    fr, _ = H.make_frame(sc, torch)
    fr.forward()
    flags, n = fr.read_status()
    fr, _ = H.make_frame(sc, torch, max_pairs=int(n * 1.05) + 4096)
    outs = fr.forward()
    assert fr.read_status()[0] == 0
    idx = rng.choice(W * Hh, 2000, replace=False)
    py, px = np.divmod(idx, W)
    p, c = orc.scene_dicts(sc)
    o = orc.render_pixels(p, c, px, py)
    g = [x.cpu().numpy() for x in outs]
    assert H.rel_l2(g[0][:, py, px].T, o["rgb"]) <= H.TOL_FWD
    assert H.rel_l2(g[1][py, px], o["depth"]) <= H.TOL_FWD
    assert H.rel_l2(g[2][py, px], o["alpha"]) <= H.TOL_FWD
    assert H.rel_l2(g[3][:, py, px].T, o["feat"]) <= H.TOL_FWD
    tg = [outs[0].clone(), outs[1].clone(), None, outs[3].clone()]
    tpx, tpy = torch.from_numpy(px).cuda(), torch.from_numpy(py).cuda()
    tg[0][:, tpy, tpx] += 0.25
    tg[1][tpy, tpx] += 0.25
    tg[3][:, tpy, tpx] += 0.25
    grads = fr.make_grads()
    loss = torch.empty(1, device="cuda")
    fr.backward_l1(outs, tg, (1.0, 1.0, 0.0, 1.0), grads, loss)
    torch.cuda.synchronize()
    assert fr.read_status()[0] == 0
    ups = [np.zeros((3, Hh, W)), np.zeros((Hh, W)), np.zeros((Hh, W)), np.zeros((C, Hh, W))]
    ups[0][:, py, px] = -1.0 / ups[0].size
    ups[1][py, px] = -1.0 / ups[1].size
    ups[3][:, py, px] = -1.0 / ups[3].size
    ob = orc.backward(p, c, dict(g_rgb=ups[0], g_depth=ups[1], g_alpha=ups[2], g_feat=ups[3]))
    amb = orc.ambiguous(p, c, H.MARGIN, px=px, py=py)
    rep = {}
    H.check_grads({k: x.cpu().numpy() for k, x in grads.items()}, ob, GRADS, flags=amb,
                  report=rep)
    print("gradients:", rep)
    # every picked element is 0.25 off in each of the three groups
    assert loss.item() == pytest.approx(3 * 0.25 * 2000 / (W * Hh), rel=1e-4)
    # the explicit-upstream adjoint (its own item kernel) with the same upstream
    g2 = fr.make_grads()
    fr.backward(*[torch.from_numpy(u.astype(np.float32)).cuda() for u in ups], g2)
    torch.cuda.synchronize()
    H.check_grads({k: x.cpu().numpy() for k, x in g2.items()}, ob, GRADS, flags=amb)
