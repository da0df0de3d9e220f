"""Pins of the oracle's visibility record (Sec. 3.2 keyframe selection, Eq. 5):
a Gaussian is visible when it is blended at some pixel while the transmittance
in front of it exceeds the threshold.  CPU only."""
import math

import numpy as np
import pytest

from paper_2504_19409_amd import scenegen as sg


def _scene(gs, W=48, H=48, f=40.0):
    """Isotropic Gaussians (x, y, z, scale, opacity) on the optical axis side."""
    n = len(gs)
    a = np.array(gs, np.float64)
    params = dict(means=a[:, :3].T.copy(),
                  log_scales=np.log(np.repeat(a[:, 3:4], 3, axis=1)).T.copy(),
                  quats=np.tile(np.array([[1.0], [0.0], [0.0], [0.0]]), (1, n)),
                  logit_opacity=np.log(a[:, 4] / (1 - a[:, 4])),
                  rgb=np.full((3, n), 0.5), feat=np.zeros((n, 1)))
    camera = dict(width=W, height=H, fx=f, fy=f, cx=W / 2, cy=H / 2,
                  viewmat=sg.identity_viewmat())
    return params, camera


def test_single_gaussian_visible_iff_alpha_reaches_min(oracle_lib):
    s, _ = oracle_lib.visibility(*_scene([(0, 0, 2.0, 0.1, 0.5)]))
    assert s.tolist() == [True]
    # opacity below alpha_min = 1/255: alpha never reaches it
    s, _ = oracle_lib.visibility(*_scene([(0, 0, 2.0, 0.1, 0.003)]))
    assert s.tolist() == [False]


def test_transmittance_in_front_of_the_gaussian(oracle_lib):
    """alpha 0.6 leaves T = 0.4 behind it, but the record uses the
    transmittance in front (1): visible at 0.5 and at 0.999, not at 1 (the
    comparison is strict)."""
    p, c = _scene([(0, 0, 2.0, 0.1, 0.6)])
    for t, want in [(0.5, True), (0.999, True), (1.0, False)]:
        s, q = oracle_lib.visibility(p, c, t_vis=t)
        assert s.tolist() == [want] and q.tolist() == [want], t


def test_occluded_behind_an_opaque_gaussian(oracle_lib):
    """A small Gaussian behind a large one clamped at alpha 0.99 over its whole
    support sees T = 0.01 in front: not visible; put in front, both are."""
    front, back = (0, 0, 2.0, 1.0, 0.999), (0, 0, 4.0, 0.05, 0.9)
    s, _ = oracle_lib.visibility(*_scene([front, back]))
    assert s.tolist() == [True, False]
    s, _ = oracle_lib.visibility(*_scene([(0, 0, 5.0, 1.0, 0.999), back]))
    assert s.tolist() == [True, True]


def test_record_shrinks_as_the_threshold_rises(oracle_lib):
    sc, _ = sg.workload_scene("tiny")
    p, c = oracle_lib.scene_dicts(sc)
    v = [oracle_lib.visibility(p, c, t_vis=t)[0] for t in (0.1, 0.5, 0.9)]
    assert np.all(v[1] <= v[0]) and np.all(v[2] <= v[1])
    assert v[0].sum() > v[1].sum() > v[2].sum() > 0


def test_bracket_is_exact_at_zero_margin(oracle_lib):
    """With no margin the sure and possible sets are the same record; a
    margin brackets it."""
    sc, _ = sg.workload_scene("tiny")
    p, c = oracle_lib.scene_dicts(sc)
    s0, q0 = oracle_lib.visibility(p, c, 0.5, 0.0)
    assert np.array_equal(s0, q0)
    s1, q1 = oracle_lib.visibility(p, c, 0.5, 1e-2)
    assert np.all(s1 <= s0) and np.all(s0 <= q1)
