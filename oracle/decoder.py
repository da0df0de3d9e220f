"""FP64 numpy reference of the learned 1x1 feature decoder (test
infrastructure only).

The paper supervises the rendered feature map F (N channels) against
foundation-model features I^f (M = 512 channels) through a lift o(.) (Eq. 11,
L1 loss).  Here o(.) is the pointwise two-layer MLP

    Y = GELU(X W1 + b1) W2 + b2,   X: [n, 16], W1: [16, 128], W2: [128, 512]

with the tanh form of GELU, 0.5 z (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))).
The HIP kernels run both products on BF16 matrix cores with FP32
accumulation; with ``bf16=True`` this reference rounds the same quantities
the kernels round (X, W1, W2, the hidden activations H, and dZ before the two
products it feeds) and computes everything else in FP64.  Gradients with
respect to the FP32 master weights pass straight through the rounding.
"""
from __future__ import annotations

import numpy as np

GELU_C = np.sqrt(2.0 / np.pi)
GELU_K = 0.044715


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    x32 = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    z = np.asarray(z, np.float64)
    return 0.5 * z * (1.0 + np.tanh(GELU_C * (z + GELU_K * z**3)))


def gelu_grad(z):
    z = np.asarray(z, np.float64)
    u = GELU_C * (z + GELU_K * z**3)
    t = np.tanh(u)
    du = GELU_C * (1.0 + 3.0 * GELU_K * z**2)
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * du


def forward(X, W1, b1, W2, b2, bf16_points=True):
    """X: [n, 16] -> dict(Z [n,128], H [n,128], Y [n,512])."""
    r = bf16 if bf16_points else (lambda a: np.asarray(a, np.float64))
    Xr, W1r, W2r = r(X), r(W1), r(W2)
    Z = Xr @ W1r + np.asarray(b1, np.float64)
    H = r(gelu(Z))
    Y = H @ W2r + np.asarray(b2, np.float64)
    return dict(Z=Z, H=H, Y=Y, Xr=Xr, W1r=W1r, W2r=W2r)


def l1_backward(X, W1, b1, W2, b2, T, scale, bf16_points=True):
    """Loss scale * sum|Y - T| and its gradients.

    Returns dict(loss, dX [n,16], dW1 [16,128], db1 [128], dW2 [128,512],
    db2 [512], Y)."""
    r = bf16 if bf16_points else (lambda a: np.asarray(a, np.float64))
    f = forward(X, W1, b1, W2, b2, bf16_points)
    Y = f["Y"]
    D = Y - np.asarray(T, np.float64)
    loss = scale * np.abs(D).sum()
    dY = scale * np.sign(D)
    dW2 = f["H"].T @ dY
    db2 = dY.sum(axis=0)
    dH = dY @ f["W2r"].T
    dZ = dH * gelu_grad(f["Z"])
    db1 = dZ.sum(axis=0)
    dZr = r(dZ)
    dW1 = f["Xr"].T @ dZr
    dX = dZr @ f["W1r"].T
    return dict(loss=loss, dX=dX, dW1=dW1, db1=db1, dW2=dW2, db2=db2, Y=Y)


def query(X, W1, b1, W2, b2, Q, gt=None):
    """Decode, then query (Eqs. 9, 10, 12), FP64 with no rounding of the
    weights or activations: Y = o(F) for X [n, 16]; logits = Y Q^T for the
    K query vectors Q [K, 512]; p = softmax over the labels; the label of the
    largest logit (the first of equal ones); with gt [n], the cross-entropy
    (1/n) sum over the pixels with gt in [0, K) of -log p(gt).
    Returns dict(logits [n, K], prob [n, K], label [n], loss)."""
    Y = forward(X, W1, b1, W2, b2, bf16_points=False)["Y"]
    logits = Y @ np.asarray(Q, np.float64).T
    m = logits.max(axis=1, keepdims=True)
    e = np.exp(logits - m)
    prob = e / e.sum(axis=1, keepdims=True)
    out = dict(logits=logits, prob=prob, label=np.argmax(logits, axis=1), loss=None)
    if gt is not None:
        gt = np.asarray(gt)
        K = logits.shape[1]
        ok = (gt >= 0) & (gt < K)
        idx = np.where(ok, gt, 0)
        nll = -np.log(prob[np.arange(len(gt)), idx])
        out["loss"] = float(np.where(ok, nll, 0.0).sum() / len(gt))
    return out
