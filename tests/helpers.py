"""Shared helpers for the GPU parity tests: device marshalling of seeded scenes,
oracle calls, and the comparison metric.

Comparison metric (the thresholds of the method are discontinuous, so a plain
max-error gate is wrong): per output group the relative L2 error
||gpu - ref|| / ||ref|| must be under the group's tolerance, and every element
must satisfy |gpu - ref| <= tol_el * (|ref| + rms(ref)) except elements the
oracle flags as decision-ambiguous (a skip / clamp / stop threshold within
``MARGIN`` relative distance), whose count is bounded.
"""
from __future__ import annotations

import numpy as np

MARGIN = 2e-5          # decisions closer than this to a threshold may flip in FP32
TOL_FWD = 1e-4         # relative L2, FP32 forward outputs
TOL_GRAD = 1e-3        # relative L2, gradients
TOL_BF16 = 1e-2        # relative L2, BF16 feature payload vs unrounded inputs


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    if nb == 0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)


def elementwise_outliers(gpu, ref, tol, mask=None):
    """Count elements outside tol * (|ref| + rms(ref)) (ignoring masked-out)."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    rms = np.sqrt(np.mean(ref**2)) if ref.size else 0.0
    bad = np.abs(gpu - ref) > tol * (np.abs(ref) + rms) + 1e-30
    if mask is not None:
        bad &= mask
    return int(bad.sum())


def scene_to_device(scene, torch, device="cuda", feat_dtype=None):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
    feat = t(scene.feat)
    if feat_dtype is not None:
        feat = feat.to(feat_dtype)
    return dict(means=t(scene.means), log_scales=t(scene.log_scales), quats=t(scene.quats),
                logit_opacity=t(scene.logit_opacity), rgb=t(scene.rgb), feat=feat,
                viewmat=t(scene.camera.viewmat.reshape(3, 4)))


def camspec(scene):
    from paper_2504_19409_amd.rasterizer import CameraSpec
    c = scene.camera
    return CameraSpec(c.width, c.height, c.fx, c.fy, c.cx, c.cy)


def make_frame(scene, torch, settings=None, max_pairs=None, feat_dtype=None, dev=None):
    from paper_2504_19409_amd.rasterizer import Frame
    d = dev or scene_to_device(scene, torch, feat_dtype=feat_dtype)
    fr = Frame(d["means"], d["log_scales"], d["quats"], d["logit_opacity"], d["rgb"],
               d["feat"] if scene.C else None, d["viewmat"], camspec(scene), settings,
               max_pairs)
    return fr, d


def oracle_settings(oracle, gsettings=None, **kw):
    """The oracle's settings matching the defaults of the library (FP64)."""
    s = oracle.default_settings(**kw)
    if gsettings is not None:
        s.render_features = int(gsettings.render_features)
    return s


def gpu_upstream(rng, W, H, C):
    from paper_2504_19409_amd import scenegen as sg
    return sg.upstream_signs(rng, W, H, C)


def targets_away(rng, out, margin=1e-3):
    """L1 targets at least ``margin`` away from the oracle's outputs ``out``
    (FP32): the sign of out - target is then the same for the GPU's output,
    which differs from the oracle's by far less than the margin."""
    out = np.asarray(out, np.float64)
    s = rng.choice([-1.0, 1.0], size=out.shape)
    return (out + s * (margin + 0.3 * np.abs(rng.normal(size=out.shape)))).astype(np.float32)
