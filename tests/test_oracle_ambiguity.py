"""Pin of the oracle's ambiguity flags (CPU).

The GPU parity tests compare gradients element by element on every Gaussian
the oracle does not flag.  The flag set must therefore contain every
Gaussian whose gradient can change when the skip (alpha_min), clamp
(alpha_max) and stop (T_min) decisions of Eqs. 2-3 are taken by a
computation whose alpha and transmittance sit within ``thr`` of the FP64
values.  Moving the thresholds themselves by up to 0.9 thr is such a
computation, seen from the other side: every decision within 0.9 thr of its
threshold may flip, every other stays.  So, for every shifted run, the
gradients of the unflagged Gaussians must be bit-identical to the unshifted
run's, and the flagged set must be needed (some flagged gradient moves).
"""
import numpy as np
import pytest

from paper_2504_19409_amd import scenegen as sg

THR = 1e-3


def _scenes():
    sc, _ = sg.workload_scene("tiny")
    dense = sg.make_scene(3000, 40, 36, 40.0, 40.0, 20.0, 18.0, 3, seed=33)
    dense.log_scales += 0.8  # every pixel saturates: many stop decisions
    return [("tiny", sc), ("dense", dense)]


SCENES = _scenes()
SHIFTS = [dict(alpha_min=+1), dict(alpha_min=-1), dict(t_min=+1), dict(t_min=-1),
          dict(alpha_max=+1), dict(alpha_max=-1), dict(alpha_min=-1, t_min=+1, alpha_max=-1),
          dict(alpha_min=+1, t_min=-1, alpha_max=+1)]


@pytest.mark.parametrize("name,sc", SCENES, ids=[n for n, _ in SCENES])
def test_unflagged_gradients_do_not_move_with_the_thresholds(oracle_lib, name, sc):
    p, c = oracle_lib.scene_dicts(sc)
    rng = np.random.default_rng(5)
    ups = sg.upstream_signs(rng, c["width"], c["height"], sc.C)
    g = dict(g_rgb=ups[0], g_depth=ups[1], g_alpha=ups[2], g_feat=ups[3])
    base = oracle_lib.backward(p, c, g)
    flags = oracle_lib.ambiguous(p, c, THR)
    assert 0 < flags.sum() < sc.P
    keep = ~flags
    moved_flagged = 0
    for sh in SHIFTS:
        st = oracle_lib.default_settings()
        for k, sgn in sh.items():
            setattr(st, k, getattr(st, k) * (1.0 + sgn * 0.9 * THR))
        b = oracle_lib.backward(p, c, g, st)
        for k in ["means", "log_scales", "quats", "rgb"]:
            np.testing.assert_array_equal(b[k][:, keep], base[k][:, keep], err_msg=(k, sh))
        np.testing.assert_array_equal(b["logit_opacity"][keep], base["logit_opacity"][keep])
        np.testing.assert_array_equal(b["feat"][keep], base["feat"][keep])
        moved_flagged += int(np.sum(b["logit_opacity"][flags] != base["logit_opacity"][flags]))
    assert moved_flagged > 0  # the flags are not vacuous


def test_flags_grow_with_the_threshold(oracle_lib):
    name, sc = SCENES[0]
    p, c = oracle_lib.scene_dicts(sc)
    f1 = oracle_lib.ambiguous(p, c, 1e-4)
    f2 = oracle_lib.ambiguous(p, c, 1e-3)
    assert np.all(f2[f1])  # monotone
    assert f2.sum() > f1.sum()
    # only listed pixels: a subset of the whole image's set
    rng = np.random.default_rng(1)
    idx = rng.choice(c["width"] * c["height"], 500, replace=False)
    py, px = np.divmod(idx, c["width"])
    f3 = oracle_lib.ambiguous(p, c, 1e-3, px=px, py=py)
    assert np.all(f2[f3])
