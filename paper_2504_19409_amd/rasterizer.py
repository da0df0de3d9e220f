"""Torch-facing binding of the HIP rasterizer.

PyTorch only supplies device memory and the stream; every stage -- preprocess,
sorts, binning, compositing, the adjoint, the pose reduction -- runs in
libgsff.so through the C ABI (include/gsff.h).  If the library is not built,
the first call raises; there is no CPU or PyTorch fallback.

Layouts (the boundary's): means / log_scales / rgb [3, P], quats [4, P]
(w, x, y, z), logit_opacity [P], feat [P, C] (float32, bfloat16 or float16),
viewmat [3, 4] world->camera, images planar [k, H, W].
"""
from __future__ import annotations

import ctypes
import dataclasses

import torch

from . import _capi

_DTYPE_CODE = {torch.float32: _capi.DTYPE_F32, torch.bfloat16: _capi.DTYPE_BF16,
               torch.float16: _capi.DTYPE_F16}


@dataclasses.dataclass
class CameraSpec:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_param(name, t, shape0=None, dtype=torch.float32):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape0 is not None and t.shape[0] != shape0:
        raise ValueError(f"{name} must have leading dimension {shape0}, got {tuple(t.shape)}")


def default_max_pairs(P: int, width: int, height: int) -> int:
    """Pair capacity used when the caller gives none: generous enough for the
    scene statistics of the synthetic workloads (about 22-30 tiles per
    Gaussian), overflow is reported through the status word."""
    tiles = ((width + 15) // 16) * ((height + 15) // 16)
    return int(min(max(64 * P, 1 << 16), P * tiles if P else 1 << 16, 0xFFFFFFF0))


class Frame:
    """Marshalled arguments and the workspace of one rendered view."""

    def __init__(self, means, log_scales, quats, logit_opacity, rgb, feat, viewmat,
                 cam: CameraSpec, settings: _capi.Settings | None = None,
                 max_pairs: int | None = None, workspace: torch.Tensor | None = None):
        P = int(means.shape[1]) if means.dim() == 2 else 0
        _check_param("means", means, 3)
        _check_param("log_scales", log_scales, 3)
        _check_param("quats", quats, 4)
        _check_param("logit_opacity", logit_opacity)
        _check_param("rgb", rgb, 3)
        _check_param("viewmat", viewmat)
        if viewmat.numel() != 12:
            raise ValueError("viewmat must hold 12 floats (3x4)")
        C = 0
        fdt = _capi.DTYPE_F32
        if feat is not None and feat.numel() > 0:
            if feat.dtype not in _DTYPE_CODE:
                raise ValueError(f"unsupported feature dtype {feat.dtype}")
            _check_param("feat", feat, P, feat.dtype)
            C = int(feat.shape[1])
            fdt = _DTYPE_CODE[feat.dtype]
        else:
            feat = None
        self.P, self.C = P, C
        self.cam = cam
        self.device = means.device
        self.settings = settings or _capi.default_settings()
        self.max_pairs = int(max_pairs) if max_pairs is not None else default_max_pairs(
            P, cam.width, cam.height)
        self.tensors = (means, log_scales, quats, logit_opacity, rgb, feat, viewmat)
        self.g = _capi.Gaussians(P, C, fdt, means.data_ptr(), log_scales.data_ptr(),
                                 quats.data_ptr(), logit_opacity.data_ptr(), rgb.data_ptr(),
                                 0 if feat is None else feat.data_ptr())
        self.c = _capi.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy,
                              viewmat.data_ptr())
        self.ws_bytes = _capi.workspace_size(P, C, self.max_pairs, cam.width, cam.height)
        if workspace is None or workspace.numel() < self.ws_bytes:
            # 256-byte alignment: the caching allocator hands out 512-byte aligned blocks
            workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        if workspace.data_ptr() % 256:
            raise ValueError("workspace must be 256-byte aligned")
        self.ws = workspace
        self.layout = _capi.workspace_layout(P, C, self.max_pairs, cam.width, cam.height)

    # -- argument tuples -------------------------------------------------
    def _head(self):
        return (ctypes.byref(self.g), ctypes.byref(self.c), ctypes.byref(self.settings),
                ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes, self.max_pairs)

    def call_stage(self, name: str):
        L = _capi.load()
        _capi.check(getattr(L, name)(*self._head(), _stream()), name)

    def alloc_outputs(self, out_feat_dtype=torch.float32):
        H, W = self.cam.height, self.cam.width
        dev = self.device
        rgb = torch.empty((3, H, W), dtype=torch.float32, device=dev)
        depth = torch.empty((H, W), dtype=torch.float32, device=dev)
        alpha = torch.empty((H, W), dtype=torch.float32, device=dev)
        feat = torch.empty((self.C, H, W), dtype=out_feat_dtype, device=dev)
        return rgb, depth, alpha, feat

    def composite_fwd(self, outs, out_feat_dtype=torch.float32):
        rgb, depth, alpha, feat = outs
        L = _capi.load()
        _capi.check(L.gsff_composite_fwd(*self._head(), _ptr(rgb), _ptr(depth), _ptr(alpha),
                                         _ptr(feat) if self.C else None,
                                         _DTYPE_CODE[out_feat_dtype], _stream()),
                    "gsff_composite_fwd")

    def forward(self, out_feat_dtype=torch.float32, outs=None):
        """outs[3] may be None when the settings turn features off."""
        outs = outs or self.alloc_outputs(out_feat_dtype)
        rgb, depth, alpha, feat = outs
        L = _capi.load()
        _capi.check(L.gsff_forward(*self._head(), _ptr(rgb), _ptr(depth), _ptr(alpha),
                                   _ptr(feat) if self.C else None,
                                   _DTYPE_CODE[out_feat_dtype], _stream()), "gsff_forward")
        return outs

    def make_grads(self, need=("means", "log_scales", "quats", "logit_opacity", "rgb", "feat",
                               "pose")):
        P, C, dev = self.P, self.C, self.device
        shapes = dict(means=(3, P), log_scales=(3, P), quats=(4, P), logit_opacity=(P,),
                      rgb=(3, P), feat=(P, C), pose=(6,))
        out = {}
        for k in need:
            if k == "feat" and C == 0:
                continue
            out[k] = torch.empty(shapes[k], dtype=torch.float32, device=dev)
        return out

    def _grads_struct(self, grads):
        return _capi.Grads(*[grads[k].data_ptr() if grads.get(k) is not None else None
                             for k in ("means", "log_scales", "quats", "logit_opacity", "rgb",
                                       "feat", "pose")])

    def backward(self, g_rgb, g_depth, g_alpha, g_feat, grads, accumulate=False):
        gs = self._grads_struct(grads)
        L = _capi.load()
        _capi.check(L.gsff_backward(*self._head(), _ptr(g_rgb), _ptr(g_depth), _ptr(g_alpha),
                                    _ptr(g_feat), ctypes.byref(gs), int(accumulate), _stream()),
                    "gsff_backward")
        return grads

    def backward_l1(self, outs, targets, weights, grads, loss=None, accumulate=False):
        """Backward of sum_k w_k mean|out_k - target_k| over (rgb, depth, alpha,
        feat); a None target leaves its group out.  ``outs`` are this frame's
        forward outputs (float32)."""
        gs = self._grads_struct(grads)
        w = (ctypes.c_float * 4)(*[float(x) for x in weights])
        o = [(None if t is None else x) for x, t in zip(outs, targets)]
        L = _capi.load()
        _capi.check(L.gsff_backward_l1(*self._head(), *[_ptr(x) for x in o],
                                       *[_ptr(t) for t in targets], w, _ptr(loss),
                                       ctypes.byref(gs), int(accumulate), _stream()),
                    "gsff_backward_l1")
        return grads

    def visibility(self, t_vis=0.5, out=None):
        """uint8 [P]: 1 for the Gaussians the last forward blended at a pixel
        with transmittance above t_vis in front of them (Eq. 5)."""
        out = out if out is not None else torch.empty(self.P, dtype=torch.uint8,
                                                      device=self.device)
        L = _capi.load()
        _capi.check(L.gsff_visibility(*self._head(), float(t_vis), _ptr(out), _stream()),
                    "gsff_visibility")
        return out

    def backward_tracking(self, outs, t_rgb, t_depth, mask_v, mask_e, lambda_t, d_pose,
                          loss=None, accumulate=False):
        """Pose gradient of the tracking loss (Eq. 6) with the Gaussians frozen:
        lambda_t mean(m_v m_e |rgb - t_rgb|) + (1 - lambda_t) mean(m_v |depth -
        t_depth|).  Masks are uint8 [H, W] (None keeps every pixel); d_pose [6]
        receives (rho, theta)."""
        L = _capi.load()
        _capi.check(L.gsff_backward_tracking(*self._head(), _ptr(outs[0]), _ptr(outs[1]),
                                             _ptr(t_rgb), _ptr(t_depth), _ptr(mask_v),
                                             _ptr(mask_e), float(lambda_t), _ptr(loss),
                                             _ptr(d_pose), int(accumulate), _stream()),
                    "gsff_backward_tracking")
        return d_pose

    def composite_bwd_l1(self, outs, targets, weights, grads, loss=None, accumulate=False):
        """Only the compositing adjoint of backward_l1 (the preprocess adjoint
        follows with preprocess_bwd); used to time the stages separately.  It
        builds the adjoint's work items itself."""
        gs = self._grads_struct(grads)
        w = (ctypes.c_float * 4)(*[float(x) for x in weights])
        o = [(None if t is None else x) for x, t in zip(outs, targets)]
        L = _capi.load()
        _capi.check(L.gsff_composite_bwd_l1(*self._head(), *[_ptr(x) for x in o],
                                            *[_ptr(t) for t in targets], w, _ptr(loss),
                                            ctypes.byref(gs), int(accumulate), _stream()),
                    "gsff_composite_bwd_l1")

    def composite_bwd(self, g_rgb, g_depth, g_alpha, g_feat, grads, accumulate=False,
                      items=True):
        if items:
            self.call_stage("gsff_adjoint_items")
        gs = self._grads_struct(grads)
        L = _capi.load()
        _capi.check(L.gsff_composite_bwd(*self._head(), _ptr(g_rgb), _ptr(g_depth),
                                         _ptr(g_alpha), _ptr(g_feat), ctypes.byref(gs),
                                         int(accumulate), _stream()), "gsff_composite_bwd")

    def preprocess_bwd(self, grads, accumulate=False):
        gs = self._grads_struct(grads)
        L = _capi.load()
        _capi.check(L.gsff_preprocess_bwd(*self._head(), ctypes.byref(gs), int(accumulate),
                                          _stream()), "gsff_preprocess_bwd")

    def read_status(self):
        flags = ctypes.c_uint32(0)
        n = ctypes.c_int64(0)
        _capi.check(_capi.load().gsff_read_status(ctypes.c_void_p(self.ws.data_ptr()),
                                                  ctypes.byref(flags), ctypes.byref(n),
                                                  _stream()), "gsff_read_status")
        return int(flags.value), int(n.value)

    def read_checks(self):
        """The checked build's bounds-test record of this workspace (zeros in
        the release build): failures, and site / index / limit of the first."""
        return _capi.read_checks(self.ws.data_ptr(), _stream().value or 0)

    # -- workspace views (for tests and inspection) -----------------------
    def ws_view(self, field: str, dtype, count):
        off = getattr(self.layout, field)
        itemsize = torch.empty((), dtype=dtype).element_size()
        return self.ws[off:off + count * itemsize].view(dtype)


def l1_grad(x: torch.Tensor, y: torch.Tensor, scale: float, grad: torch.Tensor,
            loss: torch.Tensor | None = None):
    """grad = scale * sign(x - y); loss += scale * sum|x - y| (in the library)."""
    _capi.check(_capi.load().gsff_l1_grad(_ptr(x), _ptr(y), x.numel(), float(scale), _ptr(grad),
                                          _ptr(loss), _stream()), "gsff_l1_grad")
    return grad


# Status bits of every rasterize() call since the last reset, OR-ed together
# on the device (one int32 per device), so a call never waits for the host.
_STICKY: dict = {}


def _sticky(device) -> torch.Tensor:
    key = torch.device(device)
    if key.type == "cuda" and key.index is None:
        key = torch.device("cuda", torch.cuda.current_device())
    t = _STICKY.get(key)
    if t is None:
        t = torch.zeros(1, dtype=torch.int32, device=key)
        _STICKY[key] = t
    return t


def raster_status(device="cuda", reset: bool = False) -> int:
    """The GSFF_FLAG_* bits raised by any rasterize() call on ``device`` since
    the last reset (FLAG_PAIR_OVERFLOW: some call's pairs exceeded its
    capacity and that view rendered empty).  This read waits for the device;
    rasterize() itself never does unless asked to (check_overflow=True)."""
    t = _sticky(device)
    flags = int(t.item())
    if reset:
        t.zero_()
    return flags


class _RasterizeFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, logit_opacity, rgb, feat, pose_tangent, viewmat,
                cam, settings, max_pairs, check_overflow):
        fr = Frame(means, log_scales, quats, logit_opacity, rgb, feat, viewmat, cam, settings,
                   max_pairs)
        outs = fr.forward()
        if check_overflow:
            flags, n = fr.read_status()
            if flags & _capi.FLAG_PAIR_OVERFLOW:
                fr = Frame(means, log_scales, quats, logit_opacity, rgb, feat, viewmat, cam,
                           settings, int(n * 1.25) + 1024)
                outs = fr.forward()
        else:
            st = _sticky(fr.device)
            torch.bitwise_or(st, fr.ws_view("status", torch.int32, 1), out=st)
        ctx.frame = fr
        ctx.has_feat = fr.C > 0
        return outs

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_alpha, g_feat):
        fr: Frame = ctx.frame
        H, W = fr.cam.height, fr.cam.width
        dev = fr.device

        def prep(t, shape):
            if t is None:
                return torch.zeros(shape, dtype=torch.float32, device=dev)
            return t.to(torch.float32).contiguous()

        g_rgb = prep(g_rgb, (3, H, W))
        g_depth = prep(g_depth, (H, W))
        g_alpha = prep(g_alpha, (H, W))
        g_feat = prep(g_feat, (fr.C, H, W)) if ctx.has_feat else None
        grads = fr.make_grads()
        fr.backward(g_rgb, g_depth, g_alpha, g_feat, grads)
        feat_t = fr.tensors[5]
        dfeat = grads.get("feat")
        if feat_t is not None and dfeat is not None:
            dfeat = dfeat.to(feat_t.dtype)
        return (grads["means"], grads["log_scales"], grads["quats"], grads["logit_opacity"],
                grads["rgb"], dfeat, grads["pose"], None, None, None, None, None)


def rasterize(means, log_scales, quats, logit_opacity, rgb, feat, viewmat, cam: CameraSpec,
              pose_tangent: torch.Tensor | None = None, settings=None, max_pairs=None,
              check_overflow=False):
    """Differentiable render of (rgb [3,H,W], depth [H,W], alpha [H,W],
    feat [C,H,W]).  ``pose_tangent`` ([6], zeros, requires_grad) receives the
    gradient with respect to the left perturbation T <- Exp(delta) T at
    delta = 0 (Eq. 4); its value is not applied -- fold each optimizer step
    into ``viewmat``.

    The call never waits for the device: its workspace comes from torch's
    caching allocator and its status bits are OR-ed into a device flag that
    ``raster_status()`` reads, so forward and backward can be captured into a
    graph.  A view whose pairs exceed ``max_pairs`` (default: 64 per
    Gaussian) renders empty and raises FLAG_PAIR_OVERFLOW there.  With
    ``check_overflow=True`` the call instead reads the status at once (a host
    round trip) and renders again with the capacity the frame needed."""
    if pose_tangent is None:
        pose_tangent = torch.zeros(6, dtype=torch.float32, device=means.device)
    return _RasterizeFn.apply(means, log_scales, quats, logit_opacity, rgb, feat, pose_tangent,
                              viewmat.contiguous(), cam, settings, max_pairs, check_overflow)
