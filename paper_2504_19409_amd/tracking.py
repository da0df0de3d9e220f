"""Camera tracking on the rasterizer (Sec. 3.2): the masks of the tracking
loss (Eq. 6), the pose step on the left increment of Eq. 4, and the loop that
iterates render -> pose gradient -> pose step until the increment converges.

Every step runs in libgsff kernels on the current stream; the loop reads the
increment back to the host only every ``check_every`` iterations.
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
                   beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, delta=None):
    """viewmat [3, 4] (in place) <- Exp(delta) viewmat after one Adam step on
    d_pose; state [12] holds the moments; delta [6] receives the increment."""
    _capi.check(_capi.load().gsff_pose_adam_step(
        _ptr(viewmat), _ptr(d_pose), _ptr(state), int(step), float(lr_trans), float(lr_rot),
        float(beta1), float(beta2), float(eps), _ptr(delta), _stream()), "gsff_pose_adam_step")


def covisibility(a, b, counts=None):
    """(|a and b|, |a or b|) of two uint8 visibility records, read back."""
    counts = counts if counts is not None else torch.empty(2, dtype=torch.int32,
                                                           device=a.device)
    _capi.check(_capi.load().gsff_covisibility(_ptr(a), _ptr(b), a.numel(), _ptr(counts),
                                               _stream()), "gsff_covisibility")
    both, either = (int(x) & 0xFFFFFFFF for x in counts.cpu().tolist())
    return both, either


def is_keyframe(vis_frame, vis_keyframe, tau_thresh: float) -> bool:
    """Keyframe test of Sec. 3.2: the frame becomes a keyframe when the IoU
    of its visibility record with the last keyframe's is below tau_thresh."""
    both, either = covisibility(vis_frame, vis_keyframe)
    return (both / either if either else 1.0) < tau_thresh


@dataclass
class TrackingConfig:
    lambda_t: float = 0.9          # weight of the colour term (Eq. 6)
    edge_threshold: float = 0.01   # m_e: grey-level gradient per pixel
    vis_threshold: float = 0.5     # m_v: accumulated opacity of the first render
    lr_trans: float = 1e-3
    lr_rot: float = 3e-3
    tol_trans: float = 1e-5        # convergence: |rho| and |theta| of the increment
    tol_rot: float = 1e-5
    max_iters: int = 100
    check_every: int = 10


class Tracker:
    """Tracks one frame: ``frame`` renders at its own viewmat tensor, which the
    loop updates in place; targets are the frame's colour [3, H, W] and depth
    [H, W] images.  The loop renders without features (the tracking loss does
    not use them; skipping them is what makes tracking fast) and restores the
    frame's feature setting afterwards."""

    def __init__(self, frame: Frame, t_rgb, t_depth, cfg: TrackingConfig | None = None):
        self.fr, self.t_rgb, self.t_depth = frame, t_rgb, t_depth
        self.cfg = cfg or TrackingConfig()
        dev = frame.device
        self.viewmat = frame.tensors[-1]
        rgb, depth, alpha, _ = frame.alloc_outputs()
        self.outs = (rgb, depth, alpha, None)
        self.d_pose = torch.zeros(6, device=dev)
        self.state = torch.zeros(12, device=dev)
        self.delta = torch.zeros(6, device=dev)
        self.loss = torch.zeros(1, device=dev)
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

    def _run(self):
        cfg, fr = self.cfg, self.fr
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
                           delta=self.delta)
            if it % cfg.check_every == 0 or it == cfg.max_iters:
                d = self.delta.cpu()
                if (float(d[:3].norm()) < cfg.tol_trans and
                        float(d[3:].norm()) < cfg.tol_rot):
                    converged = True
                    break
        return it, converged, first, float(self.loss.item())
