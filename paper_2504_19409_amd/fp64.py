"""Binding of the FP64 instantiation (gsff_forward_f64 / gsff_backward_f64):
the rendering path and its adjoint in double precision, from the same device
code as the FP32 kernels for the projection, its adjoint with the pose terms
(Sec. 3.2, Eq. 4) and the adjoint's per-pair and per-tile steps.  It exists
so that central finite differences can check the adjoint; it is not a
rendering path.  Argument marshalling only: the work runs in libgsff.so.

Layouts as in rasterizer.py, all float64 device tensors: means / log_scales /
rgb [3, P], quats [4, P], logit_opacity [P], feat [P, C], viewmat [3, 4].
"""
from __future__ import annotations

import ctypes

import torch

from . import _capi

GROUPS = ("means", "log_scales", "quats", "logit_opacity", "rgb", "feat")


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(name, t):
    if t is None:
        return
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 device tensor")


class Render64:
    """One scene and camera: holds the workspace and the marshalled structs
    so repeated forwards (finite differences) and the adjoint share them."""

    def __init__(self, params: dict, viewmat: torch.Tensor, width: int, height: int,
                 fx: float, fy: float, cx: float, cy: float, settings=None):
        for k in GROUPS:
            _check(k, params.get(k))
        _check("viewmat", viewmat)
        self.params = params
        self.P = int(params["means"].shape[1])
        feat = params.get("feat")
        self.C = 0 if feat is None else int(feat.shape[1])
        self.W, self.H = int(width), int(height)
        self.st = settings or _capi.default_settings()
        self.viewmat = viewmat
        self.cam = _capi.Camera64(self.W, self.H, fx, fy, cx, cy, _p(viewmat))
        n = ctypes.c_size_t(0)
        _capi.check(_capi.load().gsff_f64_workspace_size(self.P, self.C, self.W, self.H,
                                                         ctypes.byref(n)),
                    "gsff_f64_workspace_size")
        dev = params["means"].device
        self.ws = torch.empty(int(n.value) + 256, dtype=torch.uint8, device=dev)
        off = (-self.ws.data_ptr()) % 256
        self.ws_ptr = ctypes.c_void_p(self.ws.data_ptr() + off)
        self.ws_bytes = int(n.value)

    def _scene(self):
        p = self.params
        return _capi.Gaussians64(self.P, self.C, _p(p["means"]), _p(p["log_scales"]),
                                 _p(p["quats"]), _p(p["logit_opacity"]), _p(p["rgb"]),
                                 _p(p.get("feat")) if self.C else None)

    def forward(self):
        """dict rgb [3, H, W], depth, alpha [H, W], feat [C, H, W], n [H, W] int32."""
        dev = self.params["means"].device
        H, W, C = self.H, self.W, self.C
        out = dict(rgb=torch.empty(3, H, W, dtype=torch.float64, device=dev),
                   depth=torch.empty(H, W, dtype=torch.float64, device=dev),
                   alpha=torch.empty(H, W, dtype=torch.float64, device=dev),
                   feat=torch.empty(C, H, W, dtype=torch.float64, device=dev),
                   n=torch.empty(H, W, dtype=torch.int32, device=dev))
        g = self._scene()
        _capi.check(_capi.load().gsff_forward_f64(
            ctypes.byref(g), ctypes.byref(self.cam), ctypes.byref(self.st), self.ws_ptr,
            self.ws_bytes, _p(out["rgb"]), _p(out["depth"]), _p(out["alpha"]),
            _p(out["feat"]) if C else None, _p(out["n"]), _stream()), "gsff_forward_f64")
        return out

    def backward(self, g_rgb, g_depth, g_alpha, g_feat=None):
        """Gradients (float64) of sum(g * outputs) after forward() on the same
        inputs: dict of the parameter groups plus pose [6]."""
        for k, t in (("g_rgb", g_rgb), ("g_depth", g_depth), ("g_alpha", g_alpha),
                     ("g_feat", g_feat)):
            _check(k, t)
        p = self.params
        grads = {k: torch.empty_like(p[k]) for k in GROUPS[:5]}
        grads["feat"] = torch.empty_like(p["feat"]) if self.C else None
        grads["pose"] = torch.empty(6, dtype=torch.float64, device=p["means"].device)
        gr = _capi.Grads64(*[_p(grads[k]) for k in GROUPS], _p(grads["pose"]))
        g = self._scene()
        _capi.check(_capi.load().gsff_backward_f64(
            ctypes.byref(g), ctypes.byref(self.cam), ctypes.byref(self.st), self.ws_ptr,
            self.ws_bytes, _p(g_rgb), _p(g_depth), _p(g_alpha), _p(g_feat) if self.C else None,
            ctypes.byref(gr), _stream()), "gsff_backward_f64")
        return grads
