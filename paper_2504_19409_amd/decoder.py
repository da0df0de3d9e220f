"""Torch-facing binding of the learned 1x1 feature decoder (BF16 MFMA
kernels in libgsff.so).  Argument marshalling only."""
from __future__ import annotations

import ctypes

import torch

from . import _capi

LATENT, HIDDEN, OUT = 16, 128, 512


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def workspace(n_px: int, device="cuda") -> torch.Tensor:
    n = ctypes.c_size_t(0)
    _capi.check(_capi.load().gsff_decoder_workspace_size(n_px, ctypes.byref(n)),
                "gsff_decoder_workspace_size")
    return torch.empty(int(n.value), dtype=torch.uint8, device=device)


def init_params(seed: int = 0, device="cuda"):
    """FP32 master weights, fan-in scaled normal init, zero biases."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    W1 = torch.randn(LATENT, HIDDEN, generator=g) / LATENT ** 0.5
    W2 = torch.randn(HIDDEN, OUT, generator=g) / HIDDEN ** 0.5
    return dict(W1=W1.to(device), b1=torch.zeros(HIDDEN, device=device),
                W2=W2.to(device), b2=torch.zeros(OUT, device=device))


def forward(X: torch.Tensor, params: dict, ws: torch.Tensor, out_dtype=torch.bfloat16,
            out: torch.Tensor | None = None):
    """X: bf16 [16, n_px] -> Y [512, n_px] (into ``out`` when given)."""
    assert X.dtype == torch.bfloat16 and X.is_contiguous() and X.shape[0] == LATENT
    n = X.shape[1]
    if out is not None:
        assert out.shape == (OUT, n) and out.is_contiguous()
        out_dtype = out.dtype
    Y = out if out is not None else torch.empty((OUT, n), dtype=out_dtype, device=X.device)
    code = _capi.DTYPE_BF16 if out_dtype == torch.bfloat16 else _capi.DTYPE_F32
    _capi.check(_capi.load().gsff_decoder_forward(
        _p(X), _p(params["W1"]), _p(params["b1"]), _p(params["W2"]), _p(params["b2"]), _p(Y),
        code, n, _p(ws), ws.numel(), _stream()), "gsff_decoder_forward")
    return Y


def query(X: torch.Tensor, params: dict, Q: torch.Tensor, with_prob=True, with_label=True,
          gt: torch.Tensor | None = None, ws: torch.Tensor | None = None):
    """Label probabilities [K, n_px] (Eq. 12), labels [n_px] (Eq. 10) and, with
    ground-truth labels gt [n_px] int32, the cross-entropy (Eq. 9) of the
    decoded features X bf16 [16, n_px] against queries Q [K, 512], without
    forming the 512-channel map.  Returns (prob, label, loss); absent ones None."""
    assert X.dtype == torch.bfloat16 and X.is_contiguous() and X.shape[0] == LATENT
    assert Q.dtype == torch.float32 and Q.is_contiguous() and Q.shape[1] == OUT
    n, K, dev = X.shape[1], Q.shape[0], X.device
    if ws is None:
        nb = ctypes.c_size_t(0)
        _capi.check(_capi.load().gsff_decoder_query_workspace_size(K, n, ctypes.byref(nb)),
                    "gsff_decoder_query_workspace_size")
        ws = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)
    prob = torch.empty((K, n), device=dev) if with_prob else None
    label = torch.empty(n, dtype=torch.int32, device=dev) if with_label else None
    loss = torch.empty(1, device=dev) if gt is not None else None
    _capi.check(_capi.load().gsff_decoder_query(
        _p(X), _p(params["W1"]), _p(params["b1"]), _p(params["W2"]), _p(params["b2"]), _p(Q), K,
        n, _p(prob), _p(label), _p(gt), _p(loss), _p(ws), ws.numel(), _stream()),
        "gsff_decoder_query")
    return prob, label, loss


def train_step(X: torch.Tensor, params: dict, T: torch.Tensor, ws: torch.Tensor,
               scale: float | None = None, loss: torch.Tensor | None = None):
    """Fused forward + L1 + backward.  Returns dict(dX, dW1, db1, dW2, db2)."""
    assert X.dtype == torch.bfloat16 and T.dtype == torch.bfloat16
    n = X.shape[1]
    assert T.shape == (OUT, n)
    scale = 1.0 / (OUT * n) if scale is None else scale
    dev = X.device
    g = dict(dX=torch.empty((LATENT, n), device=dev), dW1=torch.empty((LATENT, HIDDEN), device=dev),
             db1=torch.empty(HIDDEN, device=dev), dW2=torch.empty((HIDDEN, OUT), device=dev),
             db2=torch.empty(OUT, device=dev))
    _capi.check(_capi.load().gsff_decoder_train_step(
        _p(X), _p(params["W1"]), _p(params["b1"]), _p(params["W2"]), _p(params["b2"]), _p(T), n,
        float(scale), _p(loss), _p(g["dX"]), _p(g["dW1"]), _p(g["db1"]), _p(g["dW2"]),
        _p(g["db2"]), _p(ws), ws.numel(), _stream()), "gsff_decoder_train_step")
    return g
