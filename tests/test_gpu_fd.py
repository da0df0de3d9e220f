"""Finite-difference checks of the HIP adjoint itself (GPU).

The FP64 instantiation (gsff_forward_f64 / gsff_backward_f64) runs the same
device code as the FP32 kernels for the projection and its adjoint with the
pose terms (Sec. 3.2, Eq. 4) and for the compositing adjoint's per-pair and
per-tile steps.  Here:

* its forward equals the FP64 oracle's forward (same definition, Eqs. 1-3),
  and its adjoint the oracle's adjoint, to FP64 rounding;
* central differences of its forward, L = sum(g * outputs) with seeded
  upstream g (the feature term only for the feature gradient: the others
  stop at the feature map), match its adjoint element by element for every
  Gaussian parameter and, through T <- Exp(+-h e_k) T, for the six pose
  coordinates.
  A difference counts only where the oracle's decision signature (every
  skip, clamp and stop) is the same at +h, at -h and at the base point;
* feature-only upstream gives exactly zero geometry and pose gradients
  (Sec. 3.1, last paragraph).
"""
import numpy as np
import pytest

from paper_2504_19409_amd import scenegen as sg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GROUPS = ["means", "log_scales", "quats", "logit_opacity", "rgb", "feat"]


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


def _scene(seed, P=32, W=40, H=36, f=44.0, C=4):
    """Small overlapping splats (a few pixels across) over 3 x 3 tiles with
    ragged right and bottom edges, a general camera pose, depths 1.5-3.5 m."""
    rng = np.random.default_rng(seed)
    vm, _ = sg.perturbed_viewmat(rng, sg.identity_viewmat(), 0.03, 4.0)
    sc = sg.make_scene(P, W, H, f, f, W / 2, H / 2, C, seed=seed, viewmat=vm)
    sc.means[2] = 1.5 + (sc.means[2] - 1.0) * 0.5
    sc.log_scales = (sc.log_scales + 1.6).astype(np.float32)
    params = dict(means=sc.means, log_scales=sc.log_scales, quats=sc.quats,
                  logit_opacity=sc.logit_opacity, rgb=sc.rgb, feat=sc.feat)
    params = {k: np.asarray(v, np.float64) for k, v in params.items()}
    cam = dict(width=W, height=H, fx=f, fy=f, cx=W / 2, cy=H / 2,
               viewmat=np.asarray(vm, np.float64))
    return params, cam


def _upstream(rng, W, H, C, geo=True, feat=True):
    z = lambda *s: np.zeros(s)
    return dict(g_rgb=rng.normal(size=(3, H, W)) if geo else z(3, H, W),
                g_depth=rng.normal(size=(H, W)) if geo else z(H, W),
                g_alpha=rng.normal(size=(H, W)) if geo else z(H, W),
                g_feat=rng.normal(size=(C, H, W)) if feat else z(C, H, W))


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()


def _render64(params, cam):
    from paper_2504_19409_amd.fp64 import Render64
    dp = {k: _dev(v) for k, v in params.items()}
    r = Render64(dp, _dev(cam["viewmat"]), cam["width"], cam["height"], cam["fx"], cam["fy"],
                 cam["cx"], cam["cy"])
    return r, dp


def _loss_dev(out, gd, feat=True):
    """sum(g * outputs); without the feature term for the geometry and pose
    differences: the feature map's gradient reaches only the features (the
    stop-gradient of Sec. 3.1), so the adjoint's geometry gradients are those
    of the colour, depth and opacity terms alone."""
    L = ((gd["g_rgb"] * out["rgb"]).sum() + (gd["g_depth"] * out["depth"]).sum()
         + (gd["g_alpha"] * out["alpha"]).sum())
    return L + (gd["g_feat"] * out["feat"]).sum() if feat else L


def _same_settings(orc):
    """The oracle's settings with the FP32 values the library's settings
    struct holds (0.3f for dilation, 1/255f, 0.99f, 1e-4f ...): the FP64 path
    reads them from that struct, and a threshold or dilation off by a float
    rounding moves the results by about 1e-9."""
    from paper_2504_19409_amd import _capi
    s = _capi.default_settings()
    return orc.default_settings(**{k: getattr(s, k) for k in (
        "near_plane", "guard", "dilation", "alpha_min", "alpha_max", "t_min")})


def _hash(orc, params, cam):
    return orc.render(params, cam, _same_settings(orc), with_hash=True)["hash"]


@pytest.mark.parametrize("seed", [3, 4])
def test_f64_forward_and_adjoint_equal_oracle(orc, seed):
    params, cam = _scene(seed)
    W, H, C = cam["width"], cam["height"], params["feat"].shape[1]
    r, _ = _render64(params, cam)
    out = {k: v.cpu().numpy() for k, v in r.forward().items()}
    ref = orc.render(params, cam, _same_settings(orc))
    ok = ref["margin"] > 1e-9  # no decision within FP64 rounding of a threshold
    assert ok.mean() > 0.99
    assert ref["n"].max() >= 3  # overlapping splats
    for k in ("rgb", "depth", "alpha", "feat"):
        err = np.abs(out[k] - ref[k])[..., ok]
        assert np.all(err <= 1e-11 * (1 + np.abs(ref[k])[..., ok])), (k, err.max())
    assert np.array_equal(out["n"][ok], ref["n"][ok])
    if not ok.all():
        pytest.skip("a decision within rounding of its threshold: adjoint comparison skipped")
    rng = np.random.default_rng(100 + seed)
    g = _upstream(rng, W, H, C)
    gd = {k: _dev(v) for k, v in g.items()}
    an = {k: v.cpu().numpy() for k, v in r.backward(**gd).items()}
    ra = orc.backward(params, cam, g, _same_settings(orc))
    for k in GROUPS + ["pose"]:
        scale = np.abs(ra[k]).max() + 1e-300
        assert np.abs(an[k] - ra[k]).max() <= 1e-10 * scale, (k, np.abs(an[k] - ra[k]).max(),
                                                               scale)


def _compare(an, fd, rtol, what):
    m = ~np.isnan(fd)
    assert m.sum() > 0, what
    a, f = an[m], fd[m]
    scale = np.sqrt(np.mean(f ** 2)) + 1e-300
    err = np.abs(a - f)
    bad = err > rtol * (np.abs(f) + scale)
    assert not bad.any(), (what, int(bad.sum()), float(err.max()), float(scale))


@pytest.mark.parametrize("seed", [5, 6])
def test_f64_adjoint_matches_central_differences(orc, seed):
    params, cam = _scene(seed)
    W, H, C = cam["width"], cam["height"], params["feat"].shape[1]
    r, dp = _render64(params, cam)
    rng = np.random.default_rng(200 + seed)
    g = _upstream(rng, W, H, C)
    gd = {k: _dev(v) for k, v in g.items()}
    r.forward()
    an = {k: v.cpu().numpy() for k, v in r.backward(**gd).items()}
    h0 = _hash(orc, params, cam)
    skipped = 0
    for name in GROUPS:
        base = params[name]
        t = dp[name].view(-1)
        fd = np.full(base.shape, np.nan)
        Ls, keep = [], []
        for j in range(base.size):
            ix = np.unravel_index(j, base.shape)
            h = 1e-6 * max(1.0, abs(base[ix]))
            vals, same = [], True
            for sgn in (+1, -1):
                v = base[ix] + sgn * h
                t[j] = v
                vals.append(_loss_dev(r.forward(), gd, feat=name == "feat"))
                p2 = dict(params)
                p2[name] = base.copy()
                p2[name][ix] = v
                same = same and _hash(orc, p2, cam) == h0
            t[j] = base[ix]  # exact restore
            Ls.append(torch.stack(vals))
            keep.append((ix, h, same))
        Lh = torch.stack(Ls).cpu().numpy()
        for (ix, h, same), (lp, lm) in zip(keep, Lh):
            if same:
                fd[ix] = (lp - lm) / (2 * h)
            else:
                skipped += 1
        _compare(an[name], fd, 2e-6, name)
    assert skipped <= 4, skipped
    # pose: T <- Exp(+-h e_k) T (left perturbation, Eq. 4)
    V = np.eye(4)
    V[:3, :] = cam["viewmat"]
    fd = np.full(6, np.nan)
    h = 1e-6
    for k in range(6):
        vals, same = [], True
        for sgn in (+1, -1):
            d = np.zeros(6)
            d[k] = sgn * h
            T = sg.se3_exp(d) @ V
            r.viewmat.copy_(_dev(T[:3, :]))
            vals.append(float(_loss_dev(r.forward(), gd, feat=False)))
            same = same and _hash(orc, params, dict(cam, viewmat=T[:3, :])) == h0
        if same:
            fd[k] = (vals[0] - vals[1]) / (2 * h)
    r.viewmat.copy_(_dev(cam["viewmat"]))
    m = ~np.isnan(fd)  # a coordinate whose +-h moves a decision is left out
    assert m.sum() >= 5, fd
    np.testing.assert_allclose(an["pose"][m], fd[m], rtol=2e-6, atol=2e-6 * np.abs(fd[m]).max())


def test_f64_feature_upstream_stays_on_its_path(orc):
    params, cam = _scene(7)
    W, H, C = cam["width"], cam["height"], params["feat"].shape[1]
    r, _ = _render64(params, cam)
    r.forward()
    rng = np.random.default_rng(7)
    gd = {k: _dev(v) for k, v in _upstream(rng, W, H, C, geo=False).items()}
    an = {k: v.cpu().numpy() for k, v in r.backward(**gd).items()}
    for k in GROUPS[:5] + ["pose"]:
        assert np.all(an[k] == 0), k
    assert np.abs(an["feat"]).max() > 0
