"""C ABI contract checks that need no GPU: the HIP library loads, exports every
entry point include/gsff.h declares, and its host-only calls (sizes, layout,
defaults, argument validation) behave as documented.  Argument validation runs
before any device work, so invalid calls return without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def capi():
    from paper_2504_19409_amd import _capi
    if not os.path.exists(_capi.LIB_PATH):
        from paper_2504_19409_amd import build
        build.build()
    _capi.load()
    return _capi


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsff_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(capi):
    lib = capi.load()
    names = _declared("gsff.h")
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares a signature for each
    assert not [n for n in names if n not in capi.SIGNATURES]


def test_checked_build_loads_and_exports_the_same_abi(capi):
    """libgsff_checked.so (the sources built with GSFF_CHECKED=1) exports the
    same entry points and says which build it is; the release build says 0.
    gsff_read_checks validates its arguments before any device work."""
    if not os.path.exists(capi.CHECKED_LIB_PATH):
        from paper_2504_19409_amd import build
        build.build()
    flag = ctypes.c_int32(-1)
    assert capi.load().gsff_is_checked_build(ctypes.byref(flag)) == 0 and flag.value == 0
    with capi.checked_library() as lib:
        missing = [n for n in _declared("gsff.h") if not hasattr(lib, n)]
        assert not missing, missing
        assert lib.gsff_is_checked_build(ctypes.byref(flag)) == 0 and flag.value == 1
        assert capi.load() is lib
        out = (ctypes.c_uint32 * 4)()
        E = capi.ERR_INVALID_ARGUMENT
        assert lib.gsff_read_checks(None, out, None) == E
        assert lib.gsff_read_checks(ctypes.c_void_p(0x100000), None, None) == E
        assert lib.gsff_is_checked_build(None) == E
        # same workspace layout in both builds
        a = capi.workspace_layout(2000, 5, 24000, 64, 48)
    b = capi.workspace_layout(2000, 5, 24000, 64, 48)
    assert a.total_bytes == b.total_bytes and a.status == b.status == 0
    assert capi.load().gsff_is_checked_build(ctypes.byref(flag)) == 0 and flag.value == 0


def test_version_and_defaults(capi):
    lib = capi.load()
    a, b = ctypes.c_int32(-1), ctypes.c_int32(-1)
    assert lib.gsff_version(ctypes.byref(a), ctypes.byref(b)) == 0
    assert (a.value, b.value) >= (0, 1)
    s = capi.default_settings()
    assert s.alpha_min == pytest.approx(1 / 255)
    assert s.alpha_max == pytest.approx(0.99)
    assert s.t_min == pytest.approx(1e-4)
    assert s.dilation == pytest.approx(0.3)
    assert s.near_plane == pytest.approx(0.2)
    assert s.render_features == 1


def test_workspace_layout_consistent(capi):
    for P, C, M, W, H in [(1, 0, 16, 1, 1), (2000, 5, 24000, 64, 48),
                          (200_000, 16, 5_000_000, 640, 480), (1_000_000, 64, 40_000_000, 1200, 680)]:
        n = capi.workspace_size(P, C, M, W, H)
        lay = capi.workspace_layout(P, C, M, W, H)
        assert lay.total_bytes == n
        offs = [lay.status, lay.records, lay.rects, lay.depth_keys, lay.depth_ids,
                lay.pair_keys, lay.tile_ranges, lay.pix_T, lay.pix_end, lay.grad2d]
        assert lay.status == 0
        assert all(o % 256 == 0 for o in offs)
        assert offs == sorted(offs) and len(set(offs)) == len(offs)
        assert lay.tiles_x == (W + 15) // 16 and lay.tiles_y == (H + 15) // 16
        assert lay.rank_bits >= max(1, (P - 1).bit_length())
        # monotone in every size
        assert capi.workspace_size(P + 1, C, M, W, H) >= n
        assert capi.workspace_size(P, C + 1, M, W, H) >= n
        assert capi.workspace_size(P, C, M + 1000, W, H) >= n


def test_unrepresentable_sizes_rejected(capi):
    lib = capi.load()
    n = ctypes.c_size_t(0)
    # rank bits + tile bits > 32
    assert lib.gsff_workspace_size(1 << 24, 0, 100, 1 << 13, 1 << 13, ctypes.byref(n)) == \
        capi.ERR_INVALID_ARGUMENT
    assert lib.gsff_workspace_size(-1, 0, 100, 64, 64, ctypes.byref(n)) == capi.ERR_INVALID_ARGUMENT
    assert lib.gsff_workspace_size(10, -1, 100, 64, 64, ctypes.byref(n)) == capi.ERR_INVALID_ARGUMENT
    assert lib.gsff_workspace_size(10, 0, 100, 0, 64, ctypes.byref(n)) == capi.ERR_INVALID_ARGUMENT
    assert lib.gsff_workspace_size(10, 0, 1 << 33, 64, 64, ctypes.byref(n)) == \
        capi.ERR_INVALID_ARGUMENT
    assert b"representable" in lib.gsff_last_error()


def _args(capi, P=10, C=0, ws=0x100000, ws_bytes=1 << 30, max_pairs=1000, W=32, H=32):
    fake = 0x7F0000000000  # never dereferenced: every call below fails validation first
    g = capi.Gaussians(P, C, capi.DTYPE_F32, fake, fake, fake, fake, fake, fake if C else None)
    c = capi.Camera(W, H, 30.0, 30.0, W / 2, H / 2, fake)
    s = capi.default_settings()
    return g, c, s, ws, ws_bytes, max_pairs


def test_argument_validation(capi):
    lib = capi.load()
    E = capi.ERR_INVALID_ARGUMENT
    g, c, s, ws, nb, mp = _args(capi)
    b = ctypes.byref
    # NULL structs / workspace / outputs
    assert lib.gsff_forward(None, b(c), b(s), ws, nb, mp, 1, 1, 1, None, 0, None) == E
    assert lib.gsff_forward(b(g), b(c), b(s), None, nb, mp, 1, 1, 1, None, 0, None) == E
    assert lib.gsff_forward(b(g), b(c), b(s), ws, nb, mp, None, 1, 1, None, 0, None) == E
    # misaligned and too-small workspace
    assert lib.gsff_forward(b(g), b(c), b(s), ws + 4, nb, mp, 1, 1, 1, None, 0, None) == E
    assert lib.gsff_forward(b(g), b(c), b(s), ws, 64, mp, 1, 1, 1, None, 0, None) == E
    assert b"too small" in lib.gsff_last_error()
    # bad settings
    s2 = capi.default_settings(alpha_min=0.0)
    assert lib.gsff_forward(b(g), b(c), b(s2), ws, nb, mp, 1, 1, 1, None, 0, None) == E
    s3 = capi.default_settings(deterministic=2)
    assert lib.gsff_forward(b(g), b(c), b(s3), ws, nb, mp, 1, 1, 1, None, 0, None) == E
    assert capi.default_settings().deterministic == 0
    # features on, C > 0, but no feature output
    g2, *_ = _args(capi, C=4)
    assert lib.gsff_forward(b(g2), b(c), b(s), ws, nb, mp, 1, 1, 1, None, 0, None) == E
    # unsupported dtypes
    g3, *_ = _args(capi, C=4)
    g3.feat_dtype = 7
    assert lib.gsff_forward(b(g3), b(c), b(s), ws, nb, mp, 1, 1, 1, 1, 0, None) == \
        capi.ERR_UNSUPPORTED
    assert lib.gsff_forward(b(g2), b(c), b(s), ws, nb, mp, 1, 1, 1, 1, 9, None) == \
        capi.ERR_UNSUPPORTED
    # bad intrinsics / image
    c2 = capi.Camera(0, 32, 30.0, 30.0, 16, 16, 1)
    assert lib.gsff_forward(b(g), b(c2), b(s), ws, nb, mp, 1, 1, 1, None, 0, None) == E
    c3 = capi.Camera(32, 32, -1.0, 30.0, 16, 16, 1)
    assert lib.gsff_forward(b(g), b(c3), b(s), ws, nb, mp, 1, 1, 1, None, 0, None) == E
    # backward: missing upstream for geometry gradients
    gr = capi.Grads(1, None, None, None, None, None, None)
    assert lib.gsff_backward(b(g), b(c), b(s), ws, nb, mp, None, 1, 1, None, b(gr), 0,
                             None) == E
    assert lib.gsff_backward(b(g), b(c), b(s), ws, nb, mp, 1, 1, 1, None, None, 0, None) == E
    # l1 and status
    assert lib.gsff_l1_grad(None, None, 10, 1.0, None, None, None) == E
    assert lib.gsff_read_status(None, None, None, None) == E


def test_tracking_and_visibility_argument_validation(capi):
    """The tracking and keyframe entry points reject bad arguments on the host,
    before anything is launched."""
    lib = capi.load()
    E = capi.ERR_INVALID_ARGUMENT
    g, c, s, ws, nb, mp = _args(capi)
    b = ctypes.byref
    # tracking backward: NULL d_pose, non-finite lambda_t
    assert lib.gsff_backward_tracking(b(g), b(c), b(s), ws, nb, mp, 1, 1, 1, 1, None, None,
                                      0.9, None, None, 0, None) == E
    assert lib.gsff_backward_tracking(b(g), b(c), b(s), ws, nb, mp, 1, 1, 1, 1, None, None,
                                      float("nan"), None, 1, 0, None) == E
    # masks: bad size, missing input, negative or non-finite threshold
    assert lib.gsff_tracking_masks(1, 1, 0, 8, 0.1, 0.5, 1, 1, None) == E
    assert lib.gsff_tracking_masks(None, 1, 8, 8, 0.1, 0.5, 1, 1, None) == E
    assert lib.gsff_tracking_masks(1, None, 8, 8, 0.1, 0.5, 1, 1, None) == E
    assert lib.gsff_tracking_masks(1, 1, 8, 8, -0.1, 0.5, 1, 1, None) == E
    assert lib.gsff_tracking_masks(1, 1, 8, 8, 0.1, float("inf"), 1, 1, None) == E
    assert lib.gsff_tracking_masks(None, None, 8, 8, 0.1, 0.5, None, None, None) == capi.OK
    # pose step: NULL pointers, step < 1, betas, eps
    step = lambda *a, conv=None: lib.gsff_pose_adam_step(*a, conv, None, None, None)
    assert step(None, 1, 1, 1, 1e-3, 1e-3, 0.9, 0.999, 1e-8) == E
    assert step(1, 1, 1, 0, 1e-3, 1e-3, 0.9, 0.999, 1e-8) == E
    assert step(1, 1, 1, 1, 1e-3, 1e-3, 1.0, 0.999, 1e-8) == E
    assert step(1, 1, 1, 1, 1e-3, 1e-3, 0.9, 0.999, 0.0) == E
    bad = [capi.PoseConvergence(0, 1e-3, 1e-3), capi.PoseConvergence(5, -1.0, 1e-3),
           capi.PoseConvergence(5, 1e-3, float("nan"))]
    for cv in bad:
        assert step(1, 1, 1, 1, 1e-3, 1e-3, 0.9, 0.999, 1e-8, conv=ctypes.byref(cv)) == E
    # visibility: NULL output with P > 0, non-finite threshold
    assert lib.gsff_visibility(b(g), b(c), b(s), ws, nb, mp, 0.5, None, None) == E
    assert lib.gsff_visibility(b(g), b(c), b(s), ws, nb, mp, float("nan"), 1, None) == E
    # co-visibility: negative n, NULL inputs, NULL counts
    assert lib.gsff_covisibility(1, 1, -1, 1, None) == E
    assert lib.gsff_covisibility(None, 1, 5, 1, None) == E
    assert lib.gsff_covisibility(1, 1, 5, None, None) == E
    # decode + query without a workspace: K outside [1, 64], NULL inputs
    q = lambda K, Qp=1: lib.gsff_decoder_query_noalloc(1, 1, 1, 1, 1, Qp, K, 10, None, None,
                                                       None, None, None)
    assert q(65) == E and q(0) == E and q(5, None) == E
    assert lib.gsff_keyframe_test(1, 1, 5, 0.9, 1, None, None) == E
    assert lib.gsff_keyframe_test(1, 1, 5, float("nan"), 1, 1, None) == E
    assert lib.gsff_keyframe_test(1, 1, -1, 0.9, 1, 1, None) == E
    # Adam: more than eight groups, none, or a NULL table
    grp = (capi.AdamGroup * 9)()
    assert lib.gsff_adam_step(grp, 9, 1, 0.9, 0.999, 1e-8, None) == E
    assert lib.gsff_adam_step(grp, 0, 1, 0.9, 0.999, 1e-8, None) == E
    assert lib.gsff_adam_step(None, 1, 1, 0.9, 0.999, 1e-8, None) == E
    # regulariser: no Gaussians, no workspace
    assert lib.gsff_scale_reg(1, 0, 0.1, 1, 1 << 20, None, None, 0, None) == E
    assert lib.gsff_scale_reg(1, 10, 0.1, None, 1 << 20, None, None, 0, None) == E
    # decode + query: K out of range, labels without a loss
    assert lib.gsff_decoder_query(1, 1, 1, 1, 1, 1, 0, 10, None, None, None, None, 1 << 20,
                                  1 << 20, None) == E
    assert lib.gsff_decoder_query(1, 1, 1, 1, 1, 1, 65, 10, None, None, None, None, 1 << 20,
                                  1 << 20, None) == E
    assert lib.gsff_decoder_query(1, 1, 1, 1, 1, 1, 4, 10, None, None, 1, None, 1 << 20,
                                  1 << 20, None) == E


def test_f64_argument_validation(capi):
    """The FP64 instantiation checks its limits and pointers on the host."""
    lib = capi.load()
    E = capi.ERR_INVALID_ARGUMENT
    n = ctypes.c_size_t(0)
    assert lib.gsff_f64_workspace_size(100, 4, 64, 48, ctypes.byref(n)) == capi.OK
    assert n.value % 256 == 0 and n.value >= 100 * 8 * 8 + 64 * 48 * 12
    for P, C, W, H in [(4097, 0, 8, 8), (10, 33, 8, 8), (10, 0, 257, 8), (10, 0, 8, 0),
                       (-1, 0, 8, 8)]:
        assert lib.gsff_f64_workspace_size(P, C, W, H, ctypes.byref(n)) == E
    assert lib.gsff_f64_workspace_size(10, 0, 8, 8, None) == E
    s = capi.default_settings()
    cam = capi.Camera64(8, 8, 10.0, 10.0, 4.0, 4.0, 1)
    g = capi.Gaussians64(10, 0, 1, 1, 1, 1, 1, None)
    b = ctypes.byref
    ws, nb = 1 << 20, 1 << 20  # aligned stand-ins, never dereferenced
    out = (1, 1, 1, None, None, None)
    # too many Gaussians, missing image output, misaligned or small workspace
    big = capi.Gaussians64(5000, 0, 1, 1, 1, 1, 1, None)
    assert lib.gsff_forward_f64(b(big), b(cam), b(s), ws, nb, *out) == E
    assert lib.gsff_forward_f64(b(g), b(cam), b(s), ws, nb, None, 1, 1, None, None, None) == E
    assert lib.gsff_forward_f64(b(g), b(cam), b(s), ws + 8, nb, *out) == E
    assert lib.gsff_forward_f64(b(g), b(cam), b(s), ws, 64, *out) == E
    # features without a feature pointer or output
    gf = capi.Gaussians64(10, 4, 1, 1, 1, 1, 1, None)
    assert lib.gsff_forward_f64(b(gf), b(cam), b(s), ws, nb, *out) == E
    # camera without a view matrix, non-positive focal length
    assert lib.gsff_forward_f64(b(g), b(capi.Camera64(8, 8, 10.0, 10.0, 4.0, 4.0, None)), b(s),
                                ws, nb, *out) == E
    assert lib.gsff_forward_f64(b(g), b(capi.Camera64(8, 8, 0.0, 10.0, 4.0, 4.0, 1)), b(s),
                                ws, nb, *out) == E
    # backward: NULL upstream, NULL gradient outputs
    gr = capi.Grads64(1, 1, 1, 1, 1, None, 1)
    assert lib.gsff_backward_f64(b(g), b(cam), b(s), ws, nb, None, 1, 1, None, b(gr), None) == E
    assert lib.gsff_backward_f64(b(g), b(cam), b(s), ws, nb, 1, 1, 1, None, None, None) == E
    gr_nopose = capi.Grads64(1, 1, 1, 1, 1, None, None)
    assert lib.gsff_backward_f64(b(g), b(cam), b(s), ws, nb, 1, 1, 1, None, b(gr_nopose),
                                 None) == E
