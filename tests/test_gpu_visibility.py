"""GPU parity of the visibility record (Eq. 5) and the co-visibility counts of
the keyframe test (Sec. 3.2) through the C ABI.

The record is a set decided by floating point (alpha against alpha_min, the
transmittance against the threshold); the oracle brackets it with the FP64
decisions widened by 0.5% (sure, possible), and the GPU's set must lie
between.  0.5% covers the largest FP32 / FP64 difference of a transmittance:
one alpha_min decision taken the other way changes it by alpha_min = 0.39%.
"""
REL = 5e-3
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import helpers as H
from paper_2504_19409_amd import scenegen as sg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


def _scene(kind):
    if kind == "tiny":
        return sg.workload_scene("tiny")[0]
    if kind == "ragged":
        return sg.make_scene(3000, 70, 50, 50.0, 50.0, 35.0, 25.0, 4, seed=61)
    if kind == "rotated":
        rng = np.random.default_rng(62)
        vm, _ = sg.perturbed_viewmat(rng, sg.identity_viewmat(), 0.1, 10.0)
        return sg.make_scene(4000, 96, 64, 70.0, 70.0, 48.0, 32.0, 4, seed=62, viewmat=vm)
    if kind == "dense":
        sc = sg.make_scene(6000, 64, 64, 60.0, 60.0, 32.0, 32.0, 4, seed=63)
        sc.log_scales += 0.7
        return sc
    if kind == "frame":
        return sg.workload_scene("frame")[0]
    raise ValueError(kind)


def _check(gpu, sure, possible, P):
    assert gpu.dtype == np.uint8 and gpu.shape == (P,)
    assert set(np.unique(gpu)) <= {0, 1}
    v = gpu != 0
    assert np.all(v[sure]), int((~v & sure).sum())
    assert not np.any(v & ~possible), int((v & ~possible).sum())
    assert (possible & ~sure).sum() <= max(8, 0.08 * possible.sum())


@pytest.mark.parametrize("kind,t_vis", [("tiny", 0.5), ("ragged", 0.5), ("rotated", 0.5),
                                        ("dense", 0.5), ("tiny", 0.9), ("dense", 0.05),
                                        ("ragged", 0.0)])
def test_visibility_matches_oracle(orc, kind, t_vis):
    sc = _scene(kind)
    fr, _ = H.make_frame(sc, torch)
    fr.forward()
    vis = torch.full((sc.P,), 7, dtype=torch.uint8, device="cuda")
    fr.visibility(t_vis, out=vis)
    torch.cuda.synchronize()
    p, c = orc.scene_dicts(sc)
    sure, possible = orc.visibility(p, c, t_vis, REL)
    _check(vis.cpu().numpy(), sure, possible, sc.P)


def test_visibility_full_frame(orc):
    """The 640x480 / 200k-Gaussian frame, with the benchmark's pair capacity."""
    sc = _scene("frame")
    fr, _ = H.make_frame(sc, torch)
    fr.forward()
    flags, n = fr.read_status()
    fr, _ = H.make_frame(sc, torch, max_pairs=int(n * 1.05) + 4096)
    fr.forward()
    assert fr.read_status()[0] == 0
    vis = fr.visibility(0.5).cpu().numpy()
    p, c = orc.scene_dicts(sc)
    sure, possible = orc.visibility(p, c, 0.5, REL)
    _check(vis, sure, possible, sc.P)
    print("visible", int(vis.sum()), "of", sc.P, "sure", int(sure.sum()), "possible",
          int(possible.sum()))


def test_visibility_empty_and_culled(orc):
    sc = sg.make_scene(500, 40, 30, 30.0, 30.0, 20.0, 15.0, 4, seed=64)
    sc.means[2] = -1.0  # every Gaussian behind the camera
    fr, _ = H.make_frame(sc, torch)
    fr.forward()
    vis = fr.visibility(0.5)
    torch.cuda.synchronize()
    assert not torch.any(vis)


@pytest.mark.parametrize("n", [0, 1, 255, 257, 100_003])
def test_covisibility_counts(n):
    from paper_2504_19409_amd.tracking import covisibility
    rng = np.random.default_rng(n)
    a = (rng.random(n) < 0.3).astype(np.uint8) * rng.integers(1, 255, size=n).astype(np.uint8)
    b = (rng.random(n) < 0.5).astype(np.uint8)
    ta = torch.from_numpy(a).cuda()
    tb = torch.from_numpy(b).cuda()
    both, either = covisibility(ta, tb)
    assert both == int(((a != 0) & (b != 0)).sum())
    assert either == int(((a != 0) | (b != 0)).sum())


def test_keyframe_decision_from_two_poses():
    """The frame against itself has IoU 1 (no keyframe); a pose 40 degrees away
    shares few visible Gaussians (a keyframe at tau = 0.9)."""
    from paper_2504_19409_amd.tracking import covisibility, is_keyframe
    sc = _scene("ragged")
    fr, d = H.make_frame(sc, torch)
    fr.forward()
    v0 = fr.visibility(0.5).clone()
    assert not is_keyframe(v0, v0, 0.9)
    rng = np.random.default_rng(65)
    vm, _ = sg.perturbed_viewmat(rng, sc.camera.viewmat, 0.0, 40.0)
    d["viewmat"].copy_(torch.from_numpy(np.ascontiguousarray(vm, np.float32)))
    fr.forward()
    assert fr.read_status()[0] == 0
    v1 = fr.visibility(0.5)
    both, either = covisibility(v0, v1)
    assert 0 < either and both < either
    assert is_keyframe(v1, v0, 0.9) == (both / either < 0.9)
    # the device decision on either side of the measured IoU, and for two
    # empty records (IoU 1)
    iou = both / either
    assert is_keyframe(v1, v0, iou + 1e-3) and not is_keyframe(v1, v0, iou - 1e-3)
    empty = torch.zeros_like(v0)
    assert not is_keyframe(empty, empty, 1.0) and is_keyframe(empty, empty, 1.001)


def test_slam_passes_on_an_empty_scene():
    """No Gaussians: the visibility record is empty, the tracking gradient and
    loss are zero against any target, and the mapping passes accept the empty
    parameter set."""
    from paper_2504_19409_amd.mapping import adam_step
    sc = sg.make_scene(0, 40, 30, 40.0, 40.0, 20.0, 15.0, 3, seed=1)
    fr, _ = H.make_frame(sc, torch)
    outs = fr.forward()
    vis = fr.visibility(0.5)
    assert vis.numel() == 0
    t_rgb = torch.full((3, 30, 40), 0.5, device="cuda")
    t_depth = torch.full((30, 40), 2.0, device="cuda")
    d_pose = torch.full((6,), 3.0, device="cuda")
    loss = torch.full((1,), 3.0, device="cuda")
    fr.backward_tracking(outs, t_rgb, t_depth, None, None, 0.9, d_pose, loss)
    torch.cuda.synchronize()
    assert not torch.any(d_pose)
    # the loss still counts the empty render against the target
    assert loss.item() == pytest.approx(0.9 * 0.5 + 0.1 * 2.0, rel=1e-6)
    e = torch.empty(0, device="cuda")
    adam_step([(e, e, e, e, 1e-3)], 1)
    torch.cuda.synchronize()
