"""Pins of the tracking oracle (Sec. 3.2, Eqs. 4-5) against closed forms, a
library routine and the oracle renderer itself; CPU only."""
import numpy as np
import pytest
import scipy.linalg

from oracle import tracking as trk


def _grey_to_rgb(g):
    return np.stack([g, g, g])


def test_edge_magnitude_constant_is_zero():
    assert np.all(trk.edge_magnitude(np.full((3, 9, 11), 0.37)) == 0.0)


@pytest.mark.parametrize("a", [0.25, 1.0 / 3.0])
def test_edge_magnitude_ramp(a):
    """A ramp of slope a along x: magnitude a inside, a / 2 on the first and
    last columns (the replicated border halves the central difference); the
    same ramp along y gives the transposed map."""
    H, W = 7, 10
    x = np.arange(W, dtype=np.float64)
    g = np.tile(a * x, (H, 1))
    m = trk.edge_magnitude(_grey_to_rgb(g))
    np.testing.assert_allclose(m[:, 1:-1], a, rtol=1e-14)
    np.testing.assert_allclose(m[:, [0, -1]], a / 2, rtol=1e-14)
    mt = trk.edge_magnitude(_grey_to_rgb(g.T.copy()))
    np.testing.assert_allclose(mt, m.T, rtol=1e-14)


def test_edge_magnitude_diagonal_ramp_and_channel_mean():
    """a x + b y gives sqrt(a^2 + b^2) inside; the grey image is the mean of
    the channels, so a slope of 3a in red alone reads as a."""
    H, W = 8, 9
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    m = trk.edge_magnitude(_grey_to_rgb(0.3 * x - 0.4 * y))
    np.testing.assert_allclose(m[1:-1, 1:-1], 0.5, rtol=1e-14)
    rgb = np.zeros((3, H, W))
    rgb[0] = 3 * 0.2 * x
    np.testing.assert_allclose(trk.edge_magnitude(rgb)[1:-1, 1:-1], 0.2, rtol=1e-14)


def test_edge_magnitude_step():
    """A vertical step of height h between columns 4 and 5: h / 2 on those two
    columns, zero elsewhere; the mask at threshold h / 4 is exactly them."""
    h = 0.8
    g = np.zeros((6, 10))
    g[:, 5:] = h
    m = trk.edge_magnitude(_grey_to_rgb(g))
    expect = np.zeros_like(g)
    expect[:, 4:6] = h / 2
    np.testing.assert_allclose(m, expect, atol=1e-15)
    assert np.array_equal(trk.edge_mask(_grey_to_rgb(g), h / 4), expect > 0)


def _rand_frame(rng, H=6, W=7):
    o_c, t_c = rng.random((3, H, W)), rng.random((3, H, W))
    o_d, t_d = 1 + rng.random((H, W)), 1 + rng.random((H, W))
    return o_c, o_d, t_c, t_d


def test_tracking_upstream_special_cases():
    rng = np.random.default_rng(3)
    o_c, o_d, t_c, t_d = _rand_frame(rng)
    H, W = o_d.shape
    lam = 0.7
    g_c, g_d, _ = trk.tracking_upstream(o_c, o_d, t_c, t_d, None, None, lam)
    # no masks: the plain weighted L1 upstream
    np.testing.assert_allclose(g_c, lam / (3 * H * W) * np.sign(o_c - t_c), rtol=1e-15)
    np.testing.assert_allclose(g_d, (1 - lam) / (H * W) * np.sign(o_d - t_d), rtol=1e-15)
    # m_e removes the colour term only, m_v both
    zero = np.zeros((H, W), np.uint8)
    g_c, g_d, L = trk.tracking_upstream(o_c, o_d, t_c, t_d, None, zero, lam)
    assert not np.any(g_c) and np.any(g_d)
    assert L == pytest.approx((1 - lam) * np.abs(o_d - t_d).mean(), rel=1e-14)
    g_c, g_d, L = trk.tracking_upstream(o_c, o_d, t_c, t_d, zero, None, lam)
    assert not np.any(g_c) and not np.any(g_d) and L == 0.0


def test_tracking_upstream_is_the_loss_derivative():
    """L is piecewise linear in the outputs: a step that crosses no kink changes
    it by exactly the upstream dotted with the step."""
    rng = np.random.default_rng(4)
    o_c, o_d, t_c, t_d = _rand_frame(rng)
    mv = (rng.random(o_d.shape) < 0.6).astype(np.uint8)
    me = (rng.random(o_d.shape) < 0.6).astype(np.uint8)
    g_c, g_d, L0 = trk.tracking_upstream(o_c, o_d, t_c, t_d, mv, me, 0.8)
    dc, dd = rng.normal(size=o_c.shape), rng.normal(size=o_d.shape)
    eps = 0.5 * min(np.abs(o_c - t_c).min() / np.abs(dc).max(),
                    np.abs(o_d - t_d).min() / np.abs(dd).max())
    _, _, L1 = trk.tracking_upstream(o_c + eps * dc, o_d + eps * dd, t_c, t_d, mv, me, 0.8)
    assert (L1 - L0) / eps == pytest.approx((g_c * dc).sum() + (g_d * dd).sum(), rel=1e-9)


@pytest.mark.parametrize("scale", [0.0, 1e-9, 1e-3, 0.3, 2.5])
def test_se3_exp_matches_matrix_exponential(scale):
    rng = np.random.default_rng(int(scale * 1000) + 1)
    d = rng.normal(size=6)
    d[3:] *= scale / max(np.linalg.norm(d[3:]), 1e-300)
    X = np.zeros((4, 4))
    X[:3, :3] = trk.hat(d[3:])
    X[:3, 3] = d[:3]
    np.testing.assert_allclose(trk.se3_exp(d), scipy.linalg.expm(X), rtol=1e-12, atol=1e-14)


def test_se3_exp_first_order_is_the_perturbation_of_eq4():
    """d/de Exp(e delta) p at 0 = rho + theta x p: the increment moves a
    camera-frame point as the pose gradient of Eq. 4 assumes
    (d mu_c / d rho = I, d mu_c / d theta = -mu_c^)."""
    rng = np.random.default_rng(5)
    d, p = rng.normal(size=6), rng.normal(size=3)
    e = 1e-7
    q = (trk.se3_exp(e * d)[:3, :3] @ p + trk.se3_exp(e * d)[:3, 3] - p) / e
    np.testing.assert_allclose(q, d[:3] + np.cross(d[3:], p), rtol=1e-6)


def test_pose_adam_first_step_closed_form():
    """At step 1 from zero moments mhat = g and vhat = g^2, so the increment is
    -lr g / (|g| + eps) per component; a zero gradient leaves the pose."""
    rng = np.random.default_rng(6)
    V = trk.se3_exp(rng.normal(size=6) * 0.2)[:3, :]
    g = rng.normal(size=6)
    V1, m, v, d = trk.pose_adam_step(V, g, np.zeros(6), np.zeros(6), 1, 2e-3, 5e-3, eps=1e-8)
    lr = np.array([2e-3] * 3 + [5e-3] * 3)
    np.testing.assert_allclose(d, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)
    T = np.eye(4)
    T[:3, :] = V
    np.testing.assert_allclose(V1, (trk.se3_exp(d) @ T)[:3, :], rtol=1e-15)
    V0, _, _, d0 = trk.pose_adam_step(V, np.zeros(6), np.zeros(6), np.zeros(6), 1, 1e-3, 1e-3)
    assert not np.any(d0)
    np.testing.assert_allclose(V0, V, rtol=1e-15, atol=1e-15)


def test_pose_gradient_step_lowers_the_tracking_loss(oracle_lib):
    """With the oracle renderer: the pose gradient of the tracking loss (its
    masked upstream through the oracle adjoint) is a descent direction, so a
    small step T <- Exp(-eta g) T lowers the loss."""
    from paper_2504_19409_amd import scenegen as sg
    sc, _ = sg.workload_scene("tiny")
    p, c = oracle_lib.scene_dicts(sc)
    ref = oracle_lib.render(p, c)
    V = np.eye(4)
    V[:3, :] = c["viewmat"]
    moved = dict(c, viewmat=(trk.se3_exp(np.array([0.01, -0.005, 0.0, 0.0, 0.01, -0.005])) @ V)[:3, :])
    mv = trk.visibility_mask(ref["alpha"], 0.5)
    me = trk.edge_mask(ref["rgb"], 0.01)
    assert mv.sum() > 0 and me.sum() > 0

    def loss_and_grad(cam):
        out = oracle_lib.render(p, cam)
        g_c, g_d, L = trk.tracking_upstream(out["rgb"], out["depth"], ref["rgb"], ref["depth"],
                                            mv, me, 0.9)
        gr = oracle_lib.backward(p, cam, dict(g_rgb=g_c, g_depth=g_d,
                                              g_alpha=np.zeros_like(g_d)))
        return L, gr["pose"]

    L0, g = loss_and_grad(moved)
    assert L0 > 0 and np.linalg.norm(g) > 0
    Vm = np.eye(4)
    Vm[:3, :] = moved["viewmat"]
    eta = 1e-3 / np.linalg.norm(g)
    L1, _ = loss_and_grad(dict(c, viewmat=(trk.se3_exp(-eta * g) @ Vm)[:3, :]))
    assert L1 < L0
