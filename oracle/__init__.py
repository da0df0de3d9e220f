"""CPU FP64 oracle for the feature-field Gaussian rasterizer (test
infrastructure only).

Only ``tests/``, the smoke check and the benchmark's ``cpu_baseline`` leg use
this package.  It shares no code with the HIP path and never imports it.

* ``gsff_oracle.cpp`` -- the plain per-pixel definition (Eqs. 1-4 of the
  paper), FP64, single-threaded; wrapped here with ctypes.
* ``brute.py``        -- an independent numpy FP64 brute force (no culling at
  all), used to validate the C++ oracle on tiny scenes.
* ``decoder.py``      -- numpy FP64 reference of the 1x1 feature decoder
  (the pointwise lift o(.) of Eq. 11).

Parity of the paper-silent constants (alpha thresholds, dilation, near plane,
guard band) is unpinned by the paper: they are fixed by the stated readings and
applied identically by both sides.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsff_oracle.cpp")
_LIB = os.path.join(_HERE, "libgsff_oracle.so")

PROJ_FIELDS = ["valid", "u", "v", "conic_a", "conic_b", "conic_c", "depth", "key",
               "opacity", "rx", "ry", "sig_a", "sig_b", "sig_c"]


def build(force: bool = True) -> str:
    """Compile the oracle with the host compiler (no contraction, no fast
    math) into ``oracle/libgsff_oracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Settings(ctypes.Structure):
    _fields_ = [("near_plane", ctypes.c_double), ("guard", ctypes.c_double),
                ("dilation", ctypes.c_double), ("alpha_min", ctypes.c_double),
                ("alpha_max", ctypes.c_double), ("t_min", ctypes.c_double),
                ("render_features", ctypes.c_int32), ("pad", ctypes.c_int32)]


class _Scene(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int64), ("C", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("logit_opacity", ctypes.c_void_p),
                ("rgb", ctypes.c_void_p), ("feat", ctypes.c_void_p)]


class _Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("viewmat", ctypes.c_double * 12)]


def default_settings(render_features: bool = True, **kw) -> Settings:
    """Defaults: near 0.2, guard 1.3, dilation 0.3, alpha in [1/255, 0.99],
    stop below transmittance 1e-4."""
    s = Settings(0.2, 1.3, 0.3, 1.0 / 255.0, 0.99, 1e-4, int(bool(render_features)), 0)
    for k, v in kw.items():
        setattr(s, k, v)
    return s


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        sp, cp, stp = ctypes.POINTER(_Scene), ctypes.POINTER(_Camera), ctypes.POINTER(Settings)
        L.orc_project.argtypes = [sp, cp, stp, vp]
        L.orc_project.restype = ctypes.c_int
        L.orc_render.argtypes = [sp, cp, stp] + [vp] * 8
        L.orc_render.restype = ctypes.c_int
        L.orc_render_pixels.argtypes = [sp, cp, stp, ctypes.c_int64, vp, vp, vp]
        L.orc_render_pixels.restype = ctypes.c_int
        L.orc_visibility.argtypes = [sp, cp, stp, ctypes.c_double, ctypes.c_double, vp, vp]
        L.orc_visibility.restype = ctypes.c_int
        L.orc_backward.argtypes = [sp, cp, stp] + [vp] * 12
        L.orc_backward.restype = ctypes.c_int
        L.orc_tile_lists.argtypes = [sp, cp, stp, ctypes.c_int32, vp, vp]
        L.orc_tile_lists.restype = ctypes.c_int64
        L.orc_work_counts.argtypes = [sp, cp, stp, ctypes.c_int32, vp]
        L.orc_work_counts.restype = ctypes.c_int
        L.orc_ambiguous.argtypes = [sp, cp, stp, ctypes.c_double, ctypes.c_int64, vp, vp, vp]
        L.orc_ambiguous.restype = ctypes.c_int
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data


class _Marshal:
    """Holds FP64 copies of the scene so the pointers stay valid."""

    def __init__(self, params: dict, camera: dict):
        self.means = _f64(params["means"])
        self.log_scales = _f64(params["log_scales"])
        self.quats = _f64(params["quats"])
        self.logit = _f64(params["logit_opacity"])
        self.rgb = _f64(params["rgb"])
        P = self.means.shape[1]
        feat = params.get("feat")
        self.feat = _f64(feat) if feat is not None and np.size(feat) else None
        self.C = 0 if self.feat is None else int(self.feat.shape[1])
        self.P = P
        self.scene = _Scene(P, self.C, 0, _ptr(self.means), _ptr(self.log_scales),
                            _ptr(self.quats), _ptr(self.logit), _ptr(self.rgb),
                            _ptr(self.feat))
        vm = _f64(camera["viewmat"]).reshape(12)
        self.W, self.H = int(camera["width"]), int(camera["height"])
        self.camera = _Camera(self.W, self.H, float(camera["fx"]), float(camera["fy"]),
                              float(camera["cx"]), float(camera["cy"]),
                              (ctypes.c_double * 12)(*vm.tolist()))


def scene_dicts(scene):
    """(params, camera) dicts from a ``scenegen.Scene``."""
    params = dict(means=scene.means, log_scales=scene.log_scales, quats=scene.quats,
                  logit_opacity=scene.logit_opacity, rgb=scene.rgb, feat=scene.feat)
    cam = scene.camera
    camera = dict(width=cam.width, height=cam.height, fx=cam.fx, fy=cam.fy, cx=cam.cx,
                  cy=cam.cy, viewmat=cam.viewmat)
    return params, camera


def project(params, camera, settings=None):
    m = _Marshal(params, camera)
    st = settings or default_settings()
    out = np.zeros((m.P, len(PROJ_FIELDS)), dtype=np.float64)
    rc = lib().orc_project(ctypes.byref(m.scene), ctypes.byref(m.camera), ctypes.byref(st),
                           _ptr(out))
    if rc != 0:
        raise ValueError("orc_project failed")
    return {k: out[:, j] for j, k in enumerate(PROJ_FIELDS)}


def render(params, camera, settings=None, with_hash=False):
    m = _Marshal(params, camera)
    st = settings or default_settings()
    H, W, C = m.H, m.W, m.C
    out = dict(rgb=np.zeros((3, H, W)), depth=np.zeros((H, W)), alpha=np.zeros((H, W)),
               feat=np.zeros((C, H, W)), T=np.zeros((H, W)),
               n=np.zeros((H, W), dtype=np.int32), margin=np.zeros((H, W)))
    h = ctypes.c_uint64(0)
    rc = lib().orc_render(ctypes.byref(m.scene), ctypes.byref(m.camera), ctypes.byref(st),
                          _ptr(out["rgb"]), _ptr(out["depth"]), _ptr(out["alpha"]),
                          _ptr(out["feat"]) if C else None, _ptr(out["T"]), _ptr(out["n"]),
                          _ptr(out["margin"]), ctypes.addressof(h))
    if rc != 0:
        raise ValueError("orc_render failed")
    if with_hash:
        out["hash"] = int(h.value)
    return out


def render_pixels(params, camera, px, py, settings=None):
    """Forward at listed pixels: dict rgb [n,3], depth [n], alpha [n], feat [n,C]."""
    m = _Marshal(params, camera)
    st = settings or default_settings()
    px = np.ascontiguousarray(px, dtype=np.int32)
    py = np.ascontiguousarray(py, dtype=np.int32)
    n = px.size
    out = np.zeros((n, 5 + m.C))
    rc = lib().orc_render_pixels(ctypes.byref(m.scene), ctypes.byref(m.camera), ctypes.byref(st),
                                 n, _ptr(px), _ptr(py), _ptr(out))
    if rc != 0:
        raise ValueError("orc_render_pixels failed")
    return dict(rgb=out[:, :3], depth=out[:, 3], alpha=out[:, 4], feat=out[:, 5:])


def visibility(params, camera, t_vis=0.5, rel=0.0, settings=None):
    """Visibility record of Eq. 5 (blended at some pixel with transmittance
    above t_vis in front): (sure, possible) bool [P]; with rel = 0 both are the
    exact FP64 record, with rel > 0 they bracket any computation whose alpha
    and transmittance are within rel (relative) of the FP64 values."""
    m = _Marshal(params, camera)
    st = settings or default_settings()
    sure = np.zeros(m.P, dtype=np.uint8)
    possible = np.zeros(m.P, dtype=np.uint8)
    rc = lib().orc_visibility(ctypes.byref(m.scene), ctypes.byref(m.camera), ctypes.byref(st),
                              float(t_vis), float(rel), _ptr(sure), _ptr(possible))
    if rc != 0:
        raise ValueError("orc_visibility failed")
    return sure.astype(bool), possible.astype(bool)


def backward(params, camera, grads, settings=None):
    """grads: dict g_rgb [3,H,W], g_depth [H,W], g_alpha [H,W], g_feat [C,H,W]
    (optional).  Returns gradients of sum(g * outputs)."""
    m = _Marshal(params, camera)
    st = settings or default_settings()
    P, C = m.P, m.C
    g_rgb, g_depth, g_alpha = (_f64(grads["g_rgb"]), _f64(grads["g_depth"]),
                               _f64(grads["g_alpha"]))
    gf = grads.get("g_feat")
    g_feat = _f64(gf) if gf is not None else None
    out = dict(means=np.zeros((3, P)), log_scales=np.zeros((3, P)), quats=np.zeros((4, P)),
               logit_opacity=np.zeros(P), rgb=np.zeros((3, P)), feat=np.zeros((P, C)),
               pose=np.zeros(6), d2d=np.zeros((P, 10)))
    rc = lib().orc_backward(ctypes.byref(m.scene), ctypes.byref(m.camera), ctypes.byref(st),
                            _ptr(g_rgb), _ptr(g_depth), _ptr(g_alpha), _ptr(g_feat),
                            _ptr(out["means"]), _ptr(out["log_scales"]), _ptr(out["quats"]),
                            _ptr(out["logit_opacity"]), _ptr(out["rgb"]),
                            _ptr(out["feat"]) if C else None, _ptr(out["pose"]),
                            _ptr(out["d2d"]))
    if rc != 0:
        raise ValueError("orc_backward failed")
    return out


def tile_lists(params, camera, tile=16, settings=None):
    """Exact per-block support lists (CSR): (counts[ntiles], ids[M])."""
    m = _Marshal(params, camera)
    st = settings or default_settings()
    ntiles = ((m.W + tile - 1) // tile) * ((m.H + tile - 1) // tile)
    counts = np.zeros(ntiles, dtype=np.int64)
    L = lib()
    M = L.orc_tile_lists(ctypes.byref(m.scene), ctypes.byref(m.camera), ctypes.byref(st),
                         tile, _ptr(counts), None)
    if M < 0:
        raise ValueError("orc_tile_lists failed")
    ids = np.zeros(max(M, 1), dtype=np.int32)
    L.orc_tile_lists(ctypes.byref(m.scene), ctypes.byref(m.camera), ctypes.byref(st),
                     tile, _ptr(counts), _ptr(ids))
    return counts, ids[:M]


def work_counts(params, camera, tile=16, settings=None):
    m = _Marshal(params, camera)
    st = settings or default_settings()
    out = np.zeros(4, dtype=np.int64)
    rc = lib().orc_work_counts(ctypes.byref(m.scene), ctypes.byref(m.camera),
                               ctypes.byref(st), tile, _ptr(out))
    if rc != 0:
        raise ValueError("orc_work_counts failed")
    return dict(pairs=int(out[0]), evals=int(out[1]), tile_evals=int(out[2]),
                contribs=int(out[3]))


def ambiguous(params, camera, thr, settings=None, px=None, py=None):
    """bool [P]: the Gaussians evaluated at a pixel with a decision within
    relative distance ``thr`` of its threshold, and the one such a pixel would
    blend next after its stop (see orc_ambiguous); only the listed pixels
    when px / py are given."""
    m = _Marshal(params, camera)
    st = settings or default_settings()
    flags = np.zeros(m.P, dtype=np.uint8)
    n = 0
    if px is not None:
        px = np.ascontiguousarray(px, dtype=np.int32)
        py = np.ascontiguousarray(py, dtype=np.int32)
        n = px.size
    rc = lib().orc_ambiguous(ctypes.byref(m.scene), ctypes.byref(m.camera), ctypes.byref(st),
                             float(thr), n, _ptr(px), _ptr(py), _ptr(flags))
    if rc != 0:
        raise ValueError("orc_ambiguous failed")
    return flags.astype(bool)
