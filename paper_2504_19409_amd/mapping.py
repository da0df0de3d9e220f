"""Mapping step on the rasterizer (Sec. 3.2, Eqs. 7-8): the keyframe window's
L1 terms (colour and depth weighted lambda_m and 1 - lambda_m; a feature term
only when asked for) over its views, the scale regulariser lambda_r L_reg,
and one fused Adam step over the Gaussians' parameters, with the camera poses
frozen.

Every step runs in libgsff kernels on the current stream.
"""
from __future__ import annotations

import ctypes

import torch

from . import _capi
from .rasterizer import _ptr, _stream
from .window import KeyframeWindow


def scale_reg_workspace(P: int, device="cuda") -> torch.Tensor:
    n = ctypes.c_size_t(0)
    _capi.check(_capi.load().gsff_scale_reg_workspace_size(int(P), ctypes.byref(n)),
                "gsff_scale_reg_workspace_size")
    return torch.empty(max(int(n.value), 8), dtype=torch.uint8, device=device)


def scale_reg(log_scales, lam: float, grad=None, loss=None, accumulate=False, workspace=None):
    """lam * L_reg of log_scales [3, P] (Eq. 7) into loss [1] and its gradient
    into grad [3, P] (either may be None)."""
    P = log_scales.shape[1]
    ws = workspace if workspace is not None else scale_reg_workspace(P, log_scales.device)
    _capi.check(_capi.load().gsff_scale_reg(_ptr(log_scales), P, float(lam), _ptr(ws),
                                            ws.numel(), _ptr(grad), _ptr(loss),
                                            int(accumulate), _stream()), "gsff_scale_reg")


def adam_step(groups, step: int, beta1=0.9, beta2=0.999, eps=1e-15):
    """groups: (param, grad, m, v, lr) tuples of FP32 device tensors, up to 8."""
    arr = (_capi.AdamGroup * len(groups))()
    for q, (p, g, m, v, lr) in enumerate(groups):
        for t in (p, g, m, v):
            if t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != p.numel():
                raise ValueError("Adam groups take contiguous FP32 tensors of one size")
        arr[q] = _capi.AdamGroup(p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(),
                                 p.numel(), float(lr))
    _capi.check(_capi.load().gsff_adam_step(arr, len(groups), int(step), float(beta1),
                                            float(beta2), float(eps), _stream()),
                "gsff_adam_step")


# Learning rates per parameter group (the paper gives none; these are the
# usual 3D Gaussian splatting rates).
DEFAULT_LR = dict(means=1.6e-4, log_scales=5e-3, quats=1e-3, logit_opacity=5e-2, rgb=2.5e-3,
                  feat=1e-3)


class Mapper:
    """One mapping step (Eq. 8) = the window's forward + fused-L1 adjoint over
    its views with colour weight lambda_m and depth weight 1 - lambda_m,
    lambda_r L_reg (Eq. 7) into the log-scale gradient and the loss, and one
    Adam step on the geometry and colour groups, the poses frozen.  Eq. 8 has
    no feature term (the paper optimises the feature field after the
    geometry, Sec. 3.3): features stay out unless ``feature_weight`` > 0,
    which adds that L1 term and the feature group (FP32 payloads only).
    Every ``check_every`` steps the window's status is read and a view that
    outgrew its pair capacity raises."""

    def __init__(self, window: KeyframeWindow, lam_m: float = 0.5, lam_reg: float = 0.01,
                 feature_weight: float = 0.0, lr: dict | None = None, betas=(0.9, 0.999),
                 eps: float = 1e-15, check_every: int = 10):
        self.win, self.lam_reg, self.betas, self.eps = window, lam_reg, betas, eps
        self.check_every = check_every
        window.weights = (float(lam_m), 1.0 - float(lam_m), 0.0, float(feature_weight))
        rates = dict(DEFAULT_LR, **(lr or {}))
        params = dict(window.geom)
        if (feature_weight > 0 and window.feat is not None
                and window.feat.dtype == torch.float32):
            params["feat"] = window.feat
        self.groups = []
        for name, p in params.items():
            g = window.grads[name]
            self.groups.append((p, g, torch.zeros_like(p), torch.zeros_like(p), rates[name]))
        P = window.geom["means"].shape[1]
        self.ws = scale_reg_workspace(P, window.geom["means"].device)
        self.n = 0

    def step(self):
        win = self.win
        win.run()
        scale_reg(win.geom["log_scales"], self.lam_reg, win.grads["log_scales"], win.loss,
                  accumulate=True, workspace=self.ws)
        self.n += 1
        adam_step(self.groups, self.n, self.betas[0], self.betas[1], self.eps)
        if self.n % self.check_every == 0:
            win.check()
        return win.loss
