"""ctypes declarations of the C ABI in include/gsff.h (argument marshalling
only; every step of the computation runs in the HIP library)."""
from __future__ import annotations

import contextlib
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsff.so")
# the checked build: every data-dependent index of the rasterizer's kernels
# tested against its buffer (see checked_library)
CHECKED_LIB_PATH = os.path.join(_HERE, "libgsff_checked.so")

OK = 0
ERR_INVALID_ARGUMENT = -1
ERR_UNSUPPORTED = -2
ERR_HIP = -3
FLAG_PAIR_OVERFLOW = 1
FLAG_SORT_RECOUNT = 2
FLAG_CHECK = 4
CHECK_SITES = {1: "sort_dest", 2: "rank_id", 3: "pair_dest", 4: "tile_range", 5: "list_id",
               6: "walk", 7: "item", 8: "row", 9: "slot", 10: "reduce"}
DTYPE_F32, DTYPE_BF16, DTYPE_F16 = 0, 1, 2
TILE = 16
SUPER = 4
MAX_CHANNELS_PER_PASS = 64

_vp = ctypes.c_void_p


class Settings(ctypes.Structure):
    _fields_ = [("near_plane", ctypes.c_float), ("guard", ctypes.c_float),
                ("dilation", ctypes.c_float), ("alpha_min", ctypes.c_float),
                ("alpha_max", ctypes.c_float), ("t_min", ctypes.c_float),
                ("render_features", ctypes.c_int32), ("bin_mode", ctypes.c_int32),
                ("deterministic", ctypes.c_int32)]


class Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float), ("viewmat", _vp)]


class Gaussians(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int64), ("C", ctypes.c_int32), ("feat_dtype", ctypes.c_int32),
                ("means", _vp), ("log_scales", _vp), ("quats", _vp), ("logit_opacity", _vp),
                ("rgb", _vp), ("feat", _vp)]


class Grads(ctypes.Structure):
    _fields_ = [("means", _vp), ("log_scales", _vp), ("quats", _vp), ("logit_opacity", _vp),
                ("rgb", _vp), ("feat", _vp), ("pose", _vp)]


class WsLayout(ctypes.Structure):
    _fields_ = [("status", ctypes.c_uint64), ("records", ctypes.c_uint64),
                ("rects", ctypes.c_uint64), ("depth_keys", ctypes.c_uint64),
                ("depth_ids", ctypes.c_uint64), ("pair_keys", ctypes.c_uint64),
                ("pair_masks", ctypes.c_uint64), ("tile_ranges", ctypes.c_uint64),
                ("tile_lists", ctypes.c_uint64), ("tile_list_ranges", ctypes.c_uint64),
                ("pix_T", ctypes.c_uint64),
                ("pix_end", ctypes.c_uint64), ("grad2d", ctypes.c_uint64),
                ("total_bytes", ctypes.c_uint64), ("rank_bits", ctypes.c_int32),
                ("tiles_x", ctypes.c_int32), ("tiles_y", ctypes.c_int32),
                ("super_x", ctypes.c_int32), ("super_y", ctypes.c_int32)]


class PoseConvergence(ctypes.Structure):
    _fields_ = [("window", ctypes.c_int32), ("tol_trans", ctypes.c_float),
                ("tol_rot", ctypes.c_float)]


POSE_STATE_FLOATS = 32


class Gaussians64(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int64), ("C", ctypes.c_int32),
                ("means", _vp), ("log_scales", _vp), ("quats", _vp), ("logit_opacity", _vp),
                ("rgb", _vp), ("feat", _vp)]


class Camera64(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("viewmat", _vp)]


class Grads64(ctypes.Structure):
    _fields_ = [("means", _vp), ("log_scales", _vp), ("quats", _vp), ("logit_opacity", _vp),
                ("rgb", _vp), ("feat", _vp), ("pose", _vp)]


class AdamGroup(ctypes.Structure):
    _fields_ = [("param", _vp), ("grad", _vp), ("m", _vp), ("v", _vp), ("n", ctypes.c_int64),
                ("lr", ctypes.c_float)]


_G, _C, _S, _R = (ctypes.POINTER(Gaussians), ctypes.POINTER(Camera), ctypes.POINTER(Settings),
                  ctypes.POINTER(Grads))
_i64, _i32, _f32, _sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_float, ctypes.c_size_t

# name -> (restype, argtypes); the header's full list of entry points
SIGNATURES = {
    "gsff_version": (_i32, [ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "gsff_last_error": (ctypes.c_char_p, []),
    "gsff_is_checked_build": (_i32, [ctypes.POINTER(_i32)]),
    "gsff_set_sort_wait_limit": (_i32, [ctypes.c_uint32]),
    "gsff_read_checks": (_i32, [_vp, ctypes.POINTER(ctypes.c_uint32), _vp]),
    "gsff_default_settings": (_i32, [_S]),
    "gsff_workspace_size": (_i32, [_i64, _i32, _i64, _i32, _i32, ctypes.POINTER(_sz)]),
    "gsff_workspace_layout": (_i32, [_i64, _i32, _i64, _i32, _i32, ctypes.POINTER(WsLayout)]),
    "gsff_forward": (_i32, [_G, _C, _S, _vp, _sz, _i64, _vp, _vp, _vp, _vp, _i32, _vp]),
    "gsff_backward": (_i32, [_G, _C, _S, _vp, _sz, _i64, _vp, _vp, _vp, _vp, _R, _i32, _vp]),
    "gsff_backward_l1": (_i32, [_G, _C, _S, _vp, _sz, _i64] + [_vp] * 8
                         + [ctypes.POINTER(_f32), _vp, _R, _i32, _vp]),
    "gsff_composite_bwd_l1": (_i32, [_G, _C, _S, _vp, _sz, _i64] + [_vp] * 8
                              + [ctypes.POINTER(_f32), _vp, _R, _i32, _vp]),
    "gsff_backward_tracking": (_i32, [_G, _C, _S, _vp, _sz, _i64] + [_vp] * 6
                               + [_f32, _vp, _vp, _i32, _vp]),
    "gsff_visibility": (_i32, [_G, _C, _S, _vp, _sz, _i64, _f32, _vp, _vp]),
    "gsff_covisibility": (_i32, [_vp, _vp, _i64, _vp, _vp]),
    "gsff_scale_reg": (_i32, [_vp, _i64, _f32, _vp, _sz, _vp, _vp, _i32, _vp]),
    "gsff_scale_reg_workspace_size": (_i32, [_i64, ctypes.POINTER(_sz)]),
    "gsff_adam_step": (_i32, [ctypes.POINTER(AdamGroup), _i32, _i32, _f32, _f32, _f32, _vp]),
    "gsff_tracking_masks": (_i32, [_vp, _vp, _i32, _i32, _f32, _f32, _vp, _vp, _vp]),
    "gsff_pose_adam_step": (_i32, [_vp, _vp, _vp, _i32, _f32, _f32, _f32, _f32, _f32,
                                   ctypes.POINTER(PoseConvergence), _vp, _vp, _vp]),
    "gsff_keyframe_test": (_i32, [_vp, _vp, _i64, _f32, _vp, _vp, _vp]),
    "gsff_preprocess": (_i32, [_G, _C, _S, _vp, _sz, _i64, _vp]),
    "gsff_sort_depth": (_i32, [_G, _C, _S, _vp, _sz, _i64, _vp]),
    "gsff_bin": (_i32, [_G, _C, _S, _vp, _sz, _i64, _vp]),
    "gsff_sort_tiles": (_i32, [_G, _C, _S, _vp, _sz, _i64, _vp]),
    "gsff_tile_ranges": (_i32, [_G, _C, _S, _vp, _sz, _i64, _vp]),
    "gsff_adjoint_items": (_i32, [_G, _C, _S, _vp, _sz, _i64, _vp]),
    "gsff_composite_fwd": (_i32, [_G, _C, _S, _vp, _sz, _i64, _vp, _vp, _vp, _vp, _i32, _vp]),
    "gsff_composite_bwd": (_i32, [_G, _C, _S, _vp, _sz, _i64, _vp, _vp, _vp, _vp, _R, _i32,
                                  _vp]),
    "gsff_preprocess_bwd": (_i32, [_G, _C, _S, _vp, _sz, _i64, _R, _i32, _vp]),
    "gsff_l1_grad": (_i32, [_vp, _vp, _i64, _f32, _vp, _vp, _vp]),
    "gsff_read_status": (_i32, [_vp, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(_i64),
                                _vp]),
    "gsff_decoder_workspace_size": (_i32, [_i64, ctypes.POINTER(_sz)]),
    "gsff_decoder_query_workspace_size": (_i32, [_i32, _i64, ctypes.POINTER(_sz)]),
    "gsff_decoder_query": (_i32, [_vp] * 6 + [_i32, _i64] + [_vp] * 5 + [_sz, _vp]),
    "gsff_decoder_query_noalloc": (_i32, [_vp] * 6 + [_i32, _i64] + [_vp] * 5),
    "gsff_f64_workspace_size": (_i32, [_i64, _i32, _i32, _i32, ctypes.POINTER(_sz)]),
    "gsff_forward_f64": (_i32, [ctypes.POINTER(Gaussians64), ctypes.POINTER(Camera64), _S, _vp,
                                _sz, _vp, _vp, _vp, _vp, _vp, _vp]),
    "gsff_backward_f64": (_i32, [ctypes.POINTER(Gaussians64), ctypes.POINTER(Camera64), _S, _vp,
                                 _sz, _vp, _vp, _vp, _vp, ctypes.POINTER(Grads64), _vp]),
    "gsff_decoder_forward": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _i32, _i64, _vp, _sz, _vp]),
    "gsff_decoder_train_step": (_i32, [_vp] * 6 + [_i64, _f32] + [_vp] * 7 + [_sz, _vp]),
}

_libs: dict[str, ctypes.CDLL] = {}
_active = LIB_PATH


def load() -> ctypes.CDLL:
    """Load libgsff.so (libgsff_checked.so inside checked_library()).  Raises
    if it is missing: there is no fallback."""
    path = _active
    if path not in _libs:
        if not os.path.exists(path):
            raise RuntimeError(
                f"{path} is not built; run paper_2504_19409_amd/build.py "
                "(or __graft_entry__.build()) first")
        L = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
        _libs[path] = L
    return _libs[path]


@contextlib.contextmanager
def checked_library():
    """Route every library call made inside the block (by this module's
    wrappers, the Frame class and the rest of the package) to the checked
    build, then back to the release build.  Both can be loaded at once; a
    workspace belongs to the build whose forward filled it."""
    global _active
    prev = _active
    _active = CHECKED_LIB_PATH
    try:
        L = load()
        flag = _i32(0)
        check(L.gsff_is_checked_build(ctypes.byref(flag)), "gsff_is_checked_build")
        if flag.value != 1:
            raise RuntimeError(f"{CHECKED_LIB_PATH} is not the checked build")
        yield L
    finally:
        _active = prev


def read_checks(ws_ptr: int, stream: int = 0) -> dict:
    """The workspace's bounds-test record (checked build; zeros otherwise):
    failures, and site / index / limit of the first one."""
    out = (ctypes.c_uint32 * 4)()
    check(load().gsff_read_checks(ctypes.c_void_p(ws_ptr), out, ctypes.c_void_p(stream)),
          "gsff_read_checks")
    return {"failures": int(out[0]), "site": CHECK_SITES.get(int(out[1]), int(out[1])),
            "index": int(out[2]), "limit": int(out[3])}


class GsffError(RuntimeError):
    pass


def check(rc: int, what: str):
    if rc != OK:
        msg = load().gsff_last_error()
        raise GsffError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")


def default_settings(**kw) -> Settings:
    s = Settings()
    check(load().gsff_default_settings(ctypes.byref(s)), "gsff_default_settings")
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def workspace_size(P, C, max_pairs, width, height) -> int:
    n = _sz(0)
    check(load().gsff_workspace_size(P, C, max_pairs, width, height, ctypes.byref(n)),
          "gsff_workspace_size")
    return int(n.value)


def workspace_layout(P, C, max_pairs, width, height) -> WsLayout:
    lay = WsLayout()
    check(load().gsff_workspace_layout(P, C, max_pairs, width, height, ctypes.byref(lay)),
          "gsff_workspace_layout")
    return lay
