"""GPU parity of the BF16-MFMA decoder kernels against the FP64 decoder
reference (same BF16 rounding points), through the C ABI.

Tolerances (relative L2): 1e-3 for FP32 outputs and every gradient group
(FP32 accumulation vs FP64; a hidden activation can round to the other BF16
neighbour when FP32 and FP64 pre-activations straddle a rounding boundary),
5e-3 with a BF16 output map (one more rounding).
"""
import numpy as np
import pytest

import helpers as H
from oracle import decoder as ref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_19409_amd import _capi
    _capi.load()


def _problem(n, seed):
    from paper_2504_19409_amd import decoder as dec
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(16, n)).astype(np.float32)
    p = dec.init_params(seed)
    p["b1"] = torch.from_numpy(rng.normal(0, 0.1, 128).astype(np.float32)).cuda()
    p["b2"] = torch.from_numpy(rng.normal(0, 0.1, 512).astype(np.float32)).cuda()
    Xb = torch.from_numpy(X).cuda().to(torch.bfloat16)
    npp = {k: v.cpu().numpy().astype(np.float64) for k, v in p.items()}
    return Xb, p, npp, rng


@pytest.mark.parametrize("n", [1000, 1004, 1003, 4096])
def test_decoder_forward_parity(n):
    """Row-aligned sizes write whole 8-pixel rows (1000: a partial last
    32-pixel block; 1004: aligned for FP32 only, its last 8-pixel group
    partial); 1003 writes element by element."""
    from paper_2504_19409_amd import decoder as dec
    Xb, p, npp, _ = _problem(n, 1)
    ws = dec.workspace(n)
    Y = dec.forward(Xb, p, ws, out_dtype=torch.float32)
    Yb = dec.forward(Xb, p, ws, out_dtype=torch.bfloat16)
    torch.cuda.synchronize()
    Xn = Xb.float().cpu().numpy().astype(np.float64)
    r = ref.forward(Xn.T, npp["W1"], npp["b1"], npp["W2"], npp["b2"])["Y"].T
    assert H.rel_l2(Y.cpu().numpy(), r) <= 1e-3
    assert H.rel_l2(Yb.float().cpu().numpy(), r) <= 5e-3


@pytest.mark.parametrize("n", [1000, 4096])
def test_decoder_train_step_parity(n):
    from paper_2504_19409_amd import decoder as dec
    Xb, p, npp, rng = _problem(n, 2)
    T = rng.normal(size=(512, n)).astype(np.float32)
    Tb = torch.from_numpy(T).cuda().to(torch.bfloat16)
    ws = dec.workspace(n)
    loss = torch.zeros(1, device="cuda")
    scale = 1.0 / (512 * n)
    g = dec.train_step(Xb, p, Tb, ws, scale, loss)
    torch.cuda.synchronize()
    Xn = Xb.float().cpu().numpy().astype(np.float64)
    Tn = Tb.float().cpu().numpy().astype(np.float64)
    r = ref.l1_backward(Xn.T, npp["W1"], npp["b1"], npp["W2"], npp["b2"], Tn.T, scale)
    assert loss.item() == pytest.approx(r["loss"], rel=1e-4)
    pairs = [("dX", g["dX"], r["dX"].T), ("dW1", g["dW1"], r["dW1"]), ("db1", g["db1"], r["db1"]),
             ("dW2", g["dW2"], r["dW2"]), ("db2", g["db2"], r["db2"])]
    for name, a, b in pairs:
        assert H.rel_l2(a.cpu().numpy(), b) <= 1e-3, (name, H.rel_l2(a.cpu().numpy(), b))


def test_decoder_full_frame_sampled():
    """640x480 = 307,200 pixels, the decoder workload's frame size: forward and
    the latent gradient on sampled pixels (both are per-pixel), weight
    gradients against the full FP64 reference."""
    from paper_2504_19409_amd import decoder as dec
    n = 640 * 480
    Xb, p, npp, rng = _problem(n, 3)
    T = rng.normal(size=(512, n)).astype(np.float32)
    Tb = torch.from_numpy(T).cuda().to(torch.bfloat16)
    ws = dec.workspace(n)
    Y = dec.forward(Xb, p, ws, out_dtype=torch.float32)
    g = dec.train_step(Xb, p, Tb, ws)
    torch.cuda.synchronize()
    Xn = Xb.float().cpu().numpy().astype(np.float64)
    Tn = Tb.float().cpu().numpy().astype(np.float64)
    pick = np.sort(rng.choice(n, 2000, replace=False))
    fr = ref.forward(Xn[:, pick].T, npp["W1"], npp["b1"], npp["W2"], npp["b2"])
    assert H.rel_l2(Y.cpu().numpy()[:, pick], fr["Y"].T) <= 1e-3
    scale = 1.0 / (512 * n)
    r = ref.l1_backward(Xn.T, npp["W1"], npp["b1"], npp["W2"], npp["b2"], Tn.T, scale)
    assert H.rel_l2(g["dX"].cpu().numpy()[:, pick], r["dX"].T[:, pick]) <= 1e-3
    for name in ["dW1", "db1", "dW2", "db2"]:
        assert H.rel_l2(g[name].cpu().numpy(), r[name]) <= 1e-3, name


# ---- decode + query (Eqs. 9, 10, 12) ----------------------------------------

@pytest.mark.parametrize("n,K", [(3000, 5), (1000, 20), (257, 64), (1, 1), (640 * 480, 20)])
def test_query_matches_oracle(n, K):
    """Probabilities to 2e-5 (FP32 vs FP64, relative L2), the cross-entropy to
    1e-5; labels equal wherever the oracle's two largest logits are further
    apart than the FP32 error of a logit (3e-5 of the pixel's largest
    |logit|: a sum of 128 FP32 products through the folded weights)."""
    from paper_2504_19409_amd import decoder as dec
    Xb, p, npp, rng = _problem(n, 100 + K)
    Q = (rng.normal(size=(K, 512)) / 20).astype(np.float32)
    gt = rng.integers(-1, K, size=n).astype(np.int32)
    prob, label, loss = dec.query(Xb, p, torch.from_numpy(Q).cuda(),
                                  gt=torch.from_numpy(gt).cuda())
    torch.cuda.synchronize()
    X = Xb.float().cpu().numpy().astype(np.float64).T  # the BF16 values, exactly
    r = ref.query(X, npp["W1"], npp["b1"], npp["W2"], npp["b2"], Q.astype(np.float64), gt=gt)
    assert H.rel_l2(prob.cpu().numpy().T, r["prob"]) <= 2e-5
    assert loss.item() == pytest.approx(r["loss"], rel=1e-5)
    lg = np.sort(r["logits"], axis=1)
    scale = np.abs(r["logits"]).max(axis=1)
    clear = (lg[:, -1] - lg[:, -2]) > 3e-5 * scale if K > 1 else np.ones(n, bool)
    assert (~clear).sum() <= max(2, n // 500), int((~clear).sum())
    assert np.array_equal(label.cpu().numpy()[clear], r["label"][clear])


def test_query_outputs_are_optional():
    from paper_2504_19409_amd import decoder as dec
    Xb, p, npp, rng = _problem(500, 7)
    Q = torch.from_numpy((rng.normal(size=(3, 512)) / 20).astype(np.float32)).cuda()
    pr, lb, ls = dec.query(Xb, p, Q)
    pr2, lb2, ls2 = dec.query(Xb, p, Q, with_prob=False)
    _, lb3, _ = dec.query(Xb, p, Q, with_label=True, with_prob=True)
    torch.cuda.synchronize()
    assert ls is None and ls2 is None and pr2 is None
    assert torch.equal(lb, lb2) and torch.equal(lb, lb3)


def test_query_without_pixels():
    """n_px = 0: nothing to label, the cross-entropy is 0."""
    from paper_2504_19409_amd import decoder as dec
    p = dec.init_params(3)
    X = torch.empty((16, 0), dtype=torch.bfloat16, device="cuda")
    Q = torch.ones((4, 512), device="cuda")
    gt = torch.empty(0, dtype=torch.int32, device="cuda")
    prob, label, loss = dec.query(X, p, Q, gt=gt)
    torch.cuda.synchronize()
    assert prob.shape == (4, 0) and label.shape == (0,) and loss.item() == 0.0
