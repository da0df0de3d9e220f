"""Keyframe-window step (several views, gradients accumulated across views,
one pose gradient per view, all launches in one HIP graph) on the GPU."""
import numpy as np
import pytest

import helpers as H
from paper_2504_19409_amd import scenegen as sg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GEO = ["means", "log_scales", "quats", "logit_opacity", "rgb", "feat"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_19409_amd import _capi
    _capi.load()


def _window(P, sizes, C, seed, feat_dtype=torch.bfloat16, weights=(1.0, 1.0, 0.0, 1.0)):
    from paper_2504_19409_amd.rasterizer import CameraSpec
    from paper_2504_19409_amd.window import KeyframeWindow
    rng = np.random.default_rng(seed)
    W0, H0, f0 = sizes[0]
    sc = sg.make_scene(P, W0, H0, f0, f0, W0 / 2, H0 / 2, C, seed=seed, rng=rng)
    vms = sg.arc_viewmats(rng, len(sizes), radius=3.0, arc=2.0, jitter_deg=2.0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    geom = dict(means=t(sc.means), log_scales=t(sc.log_scales), quats=t(sc.quats),
                logit_opacity=t(sc.logit_opacity), rgb=t(sc.rgb))
    feat = t(sc.feat).to(feat_dtype)
    views, targets = [], []
    for (W, Hh, f), vm in zip(sizes, vms):
        views.append((t(vm), CameraSpec(W, Hh, f, f, W / 2, Hh / 2)))
        tr, td, tf = sg.make_targets(rng, W, Hh, C)
        targets.append([t(tr), t(td), None, t(tf)])
    win = KeyframeWindow(geom, feat, views, targets, weights)
    return win, sc, vms, rng


def test_window_graph_replay_matches_eager():
    win, *_ = _window(20_000, [(160, 120, 131.25), (240, 136, 120.0)] * 2, 32, 51)
    win.run()
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in win.grads.items()}
    ref_pose = win.pose.clone()
    ref_loss = win.loss.clone()
    win.capture()
    for rep in range(3):
        # the program's own eager work and a synchronisation between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        win.replay()
        torch.cuda.synchronize()
        for k in ref:
            assert H.rel_l2(win.grads[k].cpu().numpy(), ref[k].cpu().numpy()) <= 1e-5, (rep, k)
        assert H.rel_l2(win.pose.cpu().numpy(), ref_pose.cpu().numpy()) <= 1e-5
        assert win.loss.item() == pytest.approx(ref_loss.item(), rel=1e-5)
        del junk


def test_window_parity_vs_oracle():
    import oracle
    oracle.build(force=False)
    sizes = [(64, 48, 50.0), (96, 64, 60.0), (64, 48, 50.0), (96, 64, 60.0)]
    win, sc, vms, rng = _window(3000, sizes, 8, 52, feat_dtype=torch.float32,
                                weights=(1.0, 0.5, 0.0, 2.0))
    p, _ = oracle.scene_dicts(sc)
    cams = [dict(width=W, height=Hh, fx=f, fy=f, cx=W / 2, cy=Hh / 2, viewmat=vm)
            for (W, Hh, f), vm in zip(sizes, vms)]
    # targets kept away from the oracle's render of each view, so that no
    # sign of out - target depends on rounding; the upstream comes from the
    # oracle's render
    refs = []
    amb = np.zeros(sc.P, dtype=bool)
    for v, cam in enumerate(cams):
        r = oracle.render(p, cam)
        o = [r["rgb"], r["depth"], r["alpha"], r["feat"]]
        margin = np.where(r["margin"] < H.MARGIN, 0.05, 1e-3)
        for k in (0, 1, 3):
            win.targets[v][k].copy_(torch.from_numpy(H.targets_away(rng, o[k], margin)))
        refs.append(o)
        amb |= oracle.ambiguous(p, cam, H.MARGIN)
    win.run()
    torch.cuda.synchronize()
    total = {k: np.zeros(np.shape(p[k]) if k != "feat" else sc.feat.shape) for k in GEO}
    for v, cam in enumerate(cams):
        outs = refs[v]
        tg = win.targets[v]
        ups = [np.sign(outs[0] - tg[0].cpu().numpy()) * 1.0 / outs[0].size,
               np.sign(outs[1] - tg[1].cpu().numpy()) * 0.5 / outs[1].size,
               np.zeros_like(outs[2]),
               np.sign(outs[3] - tg[3].cpu().numpy()) * 2.0 / outs[3].size]
        ob = oracle.backward(p, cam, dict(g_rgb=ups[0], g_depth=ups[1], g_alpha=ups[2],
                                          g_feat=ups[3]))
        for k in GEO:
            total[k] += ob[k]
        H.check_grads({"pose": win.pose[v].cpu().numpy()}, ob, ["pose"])
    H.check_grads({k: win.grads[k].cpu().numpy() for k in GEO}, total, GEO, flags=amb)
