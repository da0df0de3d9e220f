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
    which differs from the oracle's by far less than the margin.  ``margin``
    may be an array broadcast against ``out`` (wider at pixels where a
    decision near its threshold may go the other way in FP32: one skipped
    Gaussian moves an output by at most alpha_min times its value)."""
    out = np.asarray(out, np.float64)
    s = rng.choice([-1.0, 1.0], size=out.shape)
    m = np.broadcast_to(np.asarray(margin, np.float64), out.shape)
    return (out + s * (m + 0.3 * np.abs(rng.normal(size=out.shape)))).astype(np.float32)


def l1_upstream(outs, targets, weights):
    """The upstream of sum_k w_k mean|out_k - target_k| formed from the
    oracle's outputs (None target: group left out) and the loss value."""
    ups, loss = [], 0.0
    for k, (x, t) in enumerate(zip(outs, targets)):
        x = np.asarray(x, np.float64)
        if t is None or weights[k] == 0.0 or x.size == 0:
            ups.append(np.zeros_like(x))
            continue
        scale = weights[k] / x.size
        ups.append(scale * np.sign(x - t))
        loss += scale * np.abs(x - t).sum()
    return ups, loss


# gradient groups: the axis that indexes Gaussians
_GAUSS_AXIS = dict(means=1, log_scales=1, quats=1, logit_opacity=0, rgb=1, feat=0)


def check_grads(gpu: dict, ref: dict, keys, flags=None, tol=TOL_GRAD, el_tol=1e-3,
                report=None):
    """Gradient parity, per group: relative L2 <= tol over every element, and
    element by element |gpu - ref| <= el_tol (|ref| + rms(ref)) on every
    Gaussian the oracle does not flag as decision-ambiguous (``flags``, bool
    [P] from ``oracle.ambiguous``; None checks every element).  The pose is
    checked element by element as well.  ``report`` (dict) receives the
    excluded count and the worst element ratio per group."""
    for k in keys:
        if k not in gpu or k not in ref:
            continue
        g = np.asarray(gpu[k], np.float64)
        r = np.asarray(ref[k], np.float64)
        if r.size == 0 or not np.any(r):
            assert not np.any(g), k
            continue
        e = rel_l2(g, r)
        assert e <= tol, (k, e)
        keep = np.ones(r.shape, dtype=bool)
        if flags is not None and k in _GAUSS_AXIS:
            f = np.asarray(flags, bool)
            keep = np.broadcast_to((~f)[None, :] if _GAUSS_AXIS[k] == 1 and r.ndim == 2
                                   else ((~f)[:, None] if r.ndim == 2 else ~f), r.shape)
        rms = np.sqrt(np.mean(r**2))
        ratio = np.abs(g - r) / (el_tol * (np.abs(r) + rms) + 1e-300)
        worst = float(ratio[keep].max()) if keep.any() else 0.0
        if report is not None:
            report[k] = dict(rel_l2=e, worst=worst,
                             excluded=int(np.sum(flags)) if flags is not None else 0)
        n_bad = int(np.sum((ratio > 1.0) & keep))
        assert n_bad == 0, (k, n_bad, worst)
