"""Camera tracking on the rasterizer (Sec. 3.2): the masks of the tracking
loss (Eq. 6), the pose step on the left increment of Eq. 4 with its
convergence test, the keyframe test, and the loop that iterates render ->
pose gradient -> pose step until the pose has converged.

Every step and every decision runs in libgsff kernels on the current stream;
the loop reads the converged flag back to the host only every
``check_every`` iterations.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _capi
from .rasterizer import Frame, _ptr, _stream


def tracking_masks(t_rgb, alpha, edge_threshold: float, vis_threshold: float,
                   mask_v=None, mask_e=None):
    """m_v (alpha > vis_threshold) and m_e (Sobel magnitude of the grey target
    > edge_threshold) as uint8 [H, W] tensors; either input may be None to
    skip its mask."""
    H, W = (alpha if alpha is not None else t_rgb[0]).shape
    dev = (alpha if alpha is not None else t_rgb).device
    if alpha is not None and mask_v is None:
        mask_v = torch.empty((H, W), dtype=torch.uint8, device=dev)
    if t_rgb is not None and mask_e is None:
        mask_e = torch.empty((H, W), dtype=torch.uint8, device=dev)
    _capi.check(_capi.load().gsff_tracking_masks(
        _ptr(t_rgb), _ptr(alpha), W, H, float(edge_threshold), float(vis_threshold),
        _ptr(mask_v if alpha is not None else None), _ptr(mask_e if t_rgb is not None else None),
        _stream()), "gsff_tracking_masks")
    return (mask_v if alpha is not None else None), (mask_e if t_rgb is not None else None)


def pose_adam_step(viewmat, d_pose, state, step: int, lr_trans: float, lr_rot: float,
                   beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, delta=None,
                   window: int = 0, tol_trans: float = 0.0, tol_rot: float = 0.0,
                   converged=None):
    """viewmat [3, 4] (in place) <- Exp(delta) viewmat after one Adam step on
    d_pose; state [POSE_STATE_FLOATS] holds the moments, the test window's
    start and the converged flag (step 1 resets it); delta [6] receives the
    increment.  window > 0 turns on the convergence test (net motion over
    every ``window`` steps below tol_trans / tol_rot), whose flag the library
    writes to converged (uint32 [1] device tensor) and keeps on the device."""
    if state.numel() < _capi.POSE_STATE_FLOATS or state.dtype != torch.float32:
        raise ValueError(f"pose state must hold {_capi.POSE_STATE_FLOATS} float32 values")
    conv = None
    if window > 0:
        conv = ctypes.byref(_capi.PoseConvergence(int(window), float(tol_trans), float(tol_rot)))
    _capi.check(_capi.load().gsff_pose_adam_step(
        _ptr(viewmat), _ptr(d_pose), _ptr(state), int(step), float(lr_trans), float(lr_rot),
        float(beta1), float(beta2), float(eps), conv, _ptr(delta), _ptr(converged), _stream()),
        "gsff_pose_adam_step")


def pose_state(device) -> torch.Tensor:
    return torch.zeros(_capi.POSE_STATE_FLOATS, dtype=torch.float32, device=device)


def covisibility(a, b, counts=None):
    """(|a and b|, |a or b|) of two uint8 visibility records, read back."""
    counts = counts if counts is not None else torch.empty(2, dtype=torch.int32,
                                                           device=a.device)
    _capi.check(_capi.load().gsff_covisibility(_ptr(a), _ptr(b), a.numel(), _ptr(counts),
                                               _stream()), "gsff_covisibility")
    both, either = (int(x) & 0xFFFFFFFF for x in counts.cpu().tolist())
    return both, either


def keyframe_test(vis_frame, vis_keyframe, tau_thresh: float, counts=None, decision=None):
    """Keyframe test of Sec. 3.2, decided on the device: decision (int32 [1]
    device tensor, returned) is 1 when the IoU of the frame's visibility
    record with the last keyframe's is below tau_thresh.  Nothing is read
    back; counts (int32 [2]) receive the intersection and union sizes."""
    dev = vis_frame.device
    counts = counts if counts is not None else torch.empty(2, dtype=torch.int32, device=dev)
    decision = decision if decision is not None else torch.empty(1, dtype=torch.int32,
                                                                 device=dev)
    _capi.check(_capi.load().gsff_keyframe_test(_ptr(vis_frame), _ptr(vis_keyframe),
                                                vis_frame.numel(), float(tau_thresh),
                                                _ptr(counts), _ptr(decision), _stream()),
                "gsff_keyframe_test")
    return decision


def is_keyframe(vis_frame, vis_keyframe, tau_thresh: float) -> bool:
    """The device's keyframe decision, read back."""
    return bool(int(keyframe_test(vis_frame, vis_keyframe, tau_thresh).item()))


@dataclass
class TrackingConfig:
    lambda_t: float = 0.9          # weight of the colour term (Eq. 6)
    edge_threshold: float = 0.01   # m_e: grey-level gradient per pixel
    vis_threshold: float = 0.5     # m_v: accumulated opacity of the first render
    lr_trans: float = 1e-3
    lr_rot: float = 3e-3
    # convergence: the net pose motion over every `window` iterations below
    # the tolerances (None: half a full-rate step, lr_trans / 2 metres and
    # lr_rot / 2 radians).  At Adam's fixed rate single increments stay near
    # a fifth of a full step even at the optimum; while the pose still
    # travels toward it, ten iterations move it by more than half a step,
    # and once it oscillates about the optimum they do not.
    window: int = 10
    tol_trans: float | None = None
    tol_rot: float | None = None
    max_iters: int = 100
    check_every: int = 10          # iterations between reads of the device flags


class Tracker:
    """Tracks one frame: ``frame`` renders at its own viewmat tensor, which the
    loop updates in place; targets are the frame's colour [3, H, W] and depth
    [H, W] images.  The loop renders without features (the tracking loss does
    not use them; skipping them is what makes tracking fast) and restores the
    frame's feature setting afterwards.  The convergence test and its
    decision run in the library; the loop reads the converged flag and the
    workspace status every ``check_every`` iterations (its only host round
    trips) and raises if a render overflowed its pair capacity."""

    def __init__(self, frame: Frame, t_rgb, t_depth, cfg: TrackingConfig | None = None,
                 history: list | None = None):
        """history: if a list, receives a device copy of the pose after every
        iteration (no host round trip)."""
        self.fr, self.t_rgb, self.t_depth = frame, t_rgb, t_depth
        self.history = history
        self.cfg = cfg or TrackingConfig()
        dev = frame.device
        self.viewmat = frame.tensors[-1]
        rgb, depth, alpha, _ = frame.alloc_outputs()
        self.outs = (rgb, depth, alpha, None)
        self.d_pose = torch.zeros(6, device=dev)
        self.state = pose_state(dev)
        self.delta = torch.zeros(6, device=dev)
        self.loss = torch.zeros(1, device=dev)
        self.converged = torch.zeros(1, dtype=torch.int32, device=dev)
        self.mask_v = self.mask_e = None

    def run(self):
        """Returns (iterations, converged, first loss, last loss); the losses
        are those of the poses the gradients were taken at."""
        st = self.fr.settings
        keep = st.render_features
        st.render_features = 0
        try:
            return self._run()
        finally:
            st.render_features = keep

    def _tolerances(self):
        c = self.cfg
        return (0.5 * c.lr_trans if c.tol_trans is None else c.tol_trans,
                0.5 * c.lr_rot if c.tol_rot is None else c.tol_rot)

    def _run(self):
        cfg, fr = self.cfg, self.fr
        tol_t, tol_r = self._tolerances()
        # m_v from the render at the starting pose, m_e from the target
        fr.forward(outs=self.outs)
        self.mask_v, self.mask_e = tracking_masks(self.t_rgb, self.outs[2], cfg.edge_threshold,
                                                  cfg.vis_threshold)
        it, converged, first = 0, False, None
        while it < cfg.max_iters:
            if it > 0:
                fr.forward(outs=self.outs)
            fr.backward_tracking(self.outs, self.t_rgb, self.t_depth, self.mask_v, self.mask_e,
                                 cfg.lambda_t, self.d_pose, self.loss)
            if it == 0:
                first = float(self.loss.item())
            it += 1
            pose_adam_step(self.viewmat, self.d_pose, self.state, it, cfg.lr_trans, cfg.lr_rot,
                           delta=self.delta, window=cfg.window, tol_trans=tol_t, tol_rot=tol_r,
                           converged=self.converged)
            if self.history is not None:
                self.history.append(self.viewmat.clone())
            if it % cfg.check_every == 0 or it == cfg.max_iters:
                flags, _ = fr.read_status()
                if flags & _capi.FLAG_PAIR_OVERFLOW:
                    raise RuntimeError("tracking render overflowed its pair capacity; "
                                       "rebuild the frame with a larger max_pairs")
                if int(self.converged.item()):
                    converged = True
                    break
        return it, converged, first, float(self.loss.item())
