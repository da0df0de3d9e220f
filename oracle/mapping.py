"""FP64 numpy oracle of the mapping support (test infrastructure only; only
``tests/`` use it).  Shares no code with the HIP path.

Sec. 3.2, mapping loss (Eqs. 7-8):

* ``scale_reg`` -- L_reg = (1/N) sum_i |s_i - sbar|_1 with s_i = exp(log
                   scale), sbar the mean scale vector, |.|_1 over the three
                   components; returns L and dL/dlog_scales (sign(0) = 0).
* ``adam``      -- one Adam step (Kingma and Ba) on a parameter array.

The regulariser's use of the activated scales, the L1 over components and
sign(0) = 0, and the optimiser (Adam), are readings where the paper gives
no detail.
"""
from __future__ import annotations

import numpy as np


def scale_reg(log_scales, lam=1.0):
    """(loss, grad [3, N]) of lam * L_reg for log_scales [3, N]."""
    s = np.exp(np.asarray(log_scales, np.float64))
    N = s.shape[1]
    d = s - s.mean(axis=1, keepdims=True)
    sg = np.sign(d)
    loss = lam * np.abs(d).sum() / N
    # d/ds_ik of (1/N) sum_j |s_jk - mean_k|: the own term and the mean's share
    grad_s = lam / N * (sg - sg.sum(axis=1, keepdims=True) / N)
    return float(loss), grad_s * s


def adam(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Returns (param', m', v')."""
    g = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * g * g
    upd = lr * (m / (1 - beta1**step)) / (np.sqrt(v / (1 - beta2**step)) + eps)
    return np.asarray(param, np.float64) - upd, m, v
