"""Pins of the decoder reference (the pointwise lift of the rendered feature
map to the 512-channel supervision space, Eq. 11):

* GELU in its published tanh form: GELU(0) = 0, GELU(x) - GELU(-x) = x
  exactly, within 1e-3 of x*Phi(x) (the erf form, via math.erf), -> x for
  large x;
* its derivative against central differences;
* the forward against a per-pixel, per-unit loop (brute force on a tiny case);
* BF16 rounding: ties to even, and identity on values already in BF16;
* the L1 backward against FP64 central differences (targets kept away from
  the outputs so no sign flips inside the step);
* straight-through rounding: on BF16-exact inputs the rounded and unrounded
  references agree up to the rounding of the hidden layer.
"""
import math

import numpy as np
import pytest

from oracle import decoder as dec


def test_gelu_identities():
    x = np.linspace(-6, 6, 1001)
    g = dec.gelu(x)
    assert dec.gelu(0.0) == 0.0
    np.testing.assert_allclose(g - dec.gelu(-x), x, rtol=0, atol=1e-13)
    phi = np.array([0.5 * v * (1 + math.erf(v / math.sqrt(2))) for v in x])
    assert np.abs(g - phi).max() < 1e-3
    assert dec.gelu(30.0) == pytest.approx(30.0, rel=1e-15)
    assert abs(dec.gelu(-30.0)) < 1e-12


def test_gelu_grad_fd():
    x = np.linspace(-5, 5, 201)
    h = 1e-6
    fd = (dec.gelu(x + h) - dec.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(dec.gelu_grad(x), fd, rtol=1e-7, atol=1e-9)


def test_bf16_rounding():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even -> 1
    assert dec.bf16(1.0 + 2.0**-8) == 1.0
    assert dec.bf16(1.0 + 3 * 2.0**-8) == 1.0 + 2.0**-6
    v = np.array([0.5, -3.25, 1.0 + 2.0**-7, 2.0**-100])
    np.testing.assert_array_equal(dec.bf16(v), v)


def _params(rng, scale=1.0):
    W1 = rng.normal(0, 0.3, (16, 128)) * scale
    b1 = rng.normal(0, 0.1, 128)
    W2 = rng.normal(0, 0.1, (128, 512)) * scale
    b2 = rng.normal(0, 0.1, 512)
    return W1, b1, W2, b2


def test_forward_matches_loop():
    rng = np.random.default_rng(0)
    X = rng.normal(size=(3, 16))
    W1, b1, W2, b2 = _params(rng)
    f = dec.forward(X, W1, b1, W2, b2, bf16_points=False)
    for n in range(3):
        h = [0.0] * 128
        for j in range(128):
            z = b1[j] + sum(X[n, k] * W1[k, j] for k in range(16))
            h[j] = 0.5 * z * (1 + math.tanh(math.sqrt(2 / math.pi) * (z + 0.044715 * z**3)))
        for c in (0, 7, 300, 511):
            y = b2[c] + sum(h[j] * W2[j, c] for j in range(128))
            assert f["Y"][n, c] == pytest.approx(y, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("bf", [False, True])
def test_l1_backward_fd(bf):
    rng = np.random.default_rng(1)
    n = 5
    X = rng.normal(size=(n, 16))
    W1, b1, W2, b2 = _params(rng)
    Y = dec.forward(X, W1, b1, W2, b2, bf16_points=False)["Y"]
    # targets at least 0.5 away from every output: the L1 sign is constant
    T = Y + rng.choice([-1.0, 1.0], size=Y.shape) * rng.uniform(0.5, 1.0, size=Y.shape)
    scale = 1.0 / Y.size
    g = dec.l1_backward(X, W1, b1, W2, b2, T, scale, bf16_points=False)

    def L(X_, W1_, b1_, W2_, b2_):
        return dec.l1_backward(X_, W1_, b1_, W2_, b2_, T, scale, bf16_points=False)["loss"]

    args = [X, W1, b1, W2, b2]
    names = ["dX", "dW1", "db1", "dW2", "db2"]
    rng2 = np.random.default_rng(2)
    for a, name in enumerate(names):
        base = args[a]
        for _ in range(6):
            idx = tuple(rng2.integers(0, s) for s in base.shape)
            h = 1e-6
            plus = [x.copy() for x in args]
            minus = [x.copy() for x in args]
            plus[a][idx] += h
            minus[a][idx] -= h
            fd = (L(*plus) - L(*minus)) / (2 * h)
            assert g[name][idx] == pytest.approx(fd, rel=1e-6, abs=1e-12), (name, idx)
    if bf:
        # rounded reference: same structure, gradients straight through the rounding
        gr = dec.l1_backward(X, W1, b1, W2, b2, T, scale, bf16_points=True)
        for name in names:
            rel = np.linalg.norm(gr[name] - g[name]) / np.linalg.norm(g[name])
            assert rel < 2e-2, name


def test_rounding_is_identity_on_bf16_inputs():
    rng = np.random.default_rng(3)
    X = dec.bf16(rng.normal(size=(4, 16)))
    W1, b1, W2, b2 = (dec.bf16(a) for a in _params(rng))
    a = dec.forward(X, W1, b1, W2, b2, bf16_points=True)
    b = dec.forward(X, W1, b1, W2, b2, bf16_points=False)
    np.testing.assert_array_equal(a["Z"], b["Z"])
    # only the hidden layer's rounding separates the two
    np.testing.assert_array_equal(a["H"], dec.bf16(b["H"]))


# ---- decode + query (Eqs. 9, 10, 12) ----------------------------------------

def _query_case(rng, n=50, K=6):
    X = rng.normal(size=(n, 16))
    W1, b1 = rng.normal(size=(16, 128)) / 4, rng.normal(size=128) * 0.1
    W2, b2 = rng.normal(size=(128, 512)) / 11, rng.normal(size=512) * 0.1
    Q = rng.normal(size=(K, 512)) / 20
    return X, W1, b1, W2, b2, Q


def test_query_unit_queries_read_decoder_channels():
    """Queries that are unit vectors e_c give the decoder's channel c as the
    logits, so the query reads the same map the decoder writes."""
    rng = np.random.default_rng(1)
    X, W1, b1, W2, b2, _ = _query_case(rng)
    chans = [0, 17, 300, 511]
    Q = np.eye(512)[chans]
    r = dec.query(X, W1, b1, W2, b2, Q)
    Y = dec.forward(X, W1, b1, W2, b2, bf16_points=False)["Y"]
    np.testing.assert_allclose(r["logits"], Y[:, chans], rtol=1e-13, atol=1e-13)
    np.testing.assert_array_equal(r["label"], np.argmax(Y[:, chans], axis=1))


def test_query_softmax_and_cross_entropy_closed_forms():
    rng = np.random.default_rng(2)
    X, W1, b1, W2, b2, Q = _query_case(rng, K=7)
    r = dec.query(X, W1, b1, W2, b2, Q)
    np.testing.assert_allclose(r["prob"].sum(axis=1), 1.0, rtol=1e-14)
    assert np.all(r["prob"] > 0)
    # one label: probability 1; equal queries: uniform, cross-entropy log K
    r1 = dec.query(X, W1, b1, W2, b2, Q[:1])
    np.testing.assert_allclose(r1["prob"], 1.0, rtol=1e-15)
    gt = rng.integers(0, 7, size=X.shape[0])
    ru = dec.query(X, W1, b1, W2, b2, np.tile(Q[:1], (7, 1)), gt=gt)
    assert ru["loss"] == pytest.approx(np.log(7.0), rel=1e-13)
    assert np.all(ru["label"] == 0)  # ties go to the first label
    # pixels whose label is out of range stay out of the sum, not of n
    gt2 = gt.copy()
    gt2[::2] = -1
    r2 = dec.query(X, W1, b1, W2, b2, np.tile(Q[:1], (7, 1)), gt=gt2)
    assert r2["loss"] == pytest.approx(np.log(7.0) * (gt2 >= 0).sum() / len(gt2), rel=1e-13)
