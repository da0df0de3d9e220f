"""Pins of the mapping oracle (Sec. 3.2, Eqs. 7-8): the scale regulariser
against closed forms and finite differences, Adam against its first-step
closed form.  CPU only."""
import numpy as np
import pytest

from oracle import mapping as omap


def test_scale_reg_equal_scales_is_flat():
    """One Gaussian is its own mean: L and the gradient vanish exactly; equal
    scales leave only the rounding of their mean."""
    L, g = omap.scale_reg(np.log([[0.05], [0.2], [0.1]]))
    assert L == 0.0 and not np.any(g)
    L, _ = omap.scale_reg(np.full((3, 7), np.log(0.05)))
    assert L <= 1e-15


def test_scale_reg_two_gaussians_closed_form():
    """Two scales a, b per component: sbar = (a + b) / 2, L = sum_k |a_k - b_k| / 2
    and dL/da_k = sign(a_k - b_k) / 2 (the two signs around the mean cancel in
    the mean's share), times a_k for the log-scale."""
    a, b = np.array([0.1, 0.3, 0.2]), np.array([0.2, 0.1, 0.25])
    ls = np.log(np.stack([a, b], axis=1))
    L, g = omap.scale_reg(ls, lam=2.0)
    assert L == pytest.approx(2.0 * np.abs(a - b).sum() / 2, rel=1e-14)
    np.testing.assert_allclose(g[:, 0], 2.0 * np.sign(a - b) / 2 * a, rtol=1e-14)
    np.testing.assert_allclose(g[:, 1], 2.0 * np.sign(b - a) / 2 * b, rtol=1e-14)


@pytest.mark.parametrize("N", [5, 40])
def test_scale_reg_matches_finite_differences(N):
    """L is smooth in the log-scales away from ties with the mean: central
    differences of L equal the gradient, the mean's dependence included."""
    rng = np.random.default_rng(N)
    ls = rng.normal(-3.0, 0.5, size=(3, N))
    _, g = omap.scale_reg(ls, lam=0.7)
    h = 1e-6
    fd = np.zeros_like(ls)
    for k in range(3):
        for i in range(N):
            e = np.zeros_like(ls)
            e[k, i] = h
            fd[k, i] = (omap.scale_reg(ls + e, 0.7)[0] - omap.scale_reg(ls - e, 0.7)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-12)


def test_adam_first_step_and_zero_gradient():
    rng = np.random.default_rng(3)
    p, g = rng.normal(size=11), rng.normal(size=11)
    p1, m, v = omap.adam(p, g, np.zeros(11), np.zeros(11), 1, 0.01, eps=1e-8)
    np.testing.assert_allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)
    p0, _, _ = omap.adam(p, np.zeros(11), np.zeros(11), np.zeros(11), 1, 0.01)
    np.testing.assert_array_equal(p0, p)
