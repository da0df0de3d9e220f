"""The learned decoder path against the method without it (GPU).

Teacher: the plain rasterizer rendering 512-channel BF16 features per
Gaussian (class-structured stand-ins for text embeddings, 32 classes).
Student: 16-channel latents rendered by the same rasterizer and lifted by the
BF16-MFMA decoder, trained on six views of an arc with this library's kernels
(latent render -> fused decoder L1 step -> feature-only rasterizer adjoint).
On two held-out views the student must reproduce the teacher's maps to a
stated error and label (Eq. 12 argmax) agreement while rendering faster and
storing 32x fewer feature bytes per Gaussian.
"""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_19409_amd import _capi
    _capi.load()


def _setup(P=60_000, W=320, H=240, f=262.5, seed=4):
    from paper_2504_19409_amd import scenegen as sg
    from paper_2504_19409_amd.distill import View, render_features
    from paper_2504_19409_amd.rasterizer import CameraSpec
    rng = np.random.default_rng(seed)
    sc = sg.make_scene(P, W, H, f, f, W / 2, H / 2, 0, seed=seed, rng=rng)
    feat, labels, q = sg.semantic_features(rng, sc.means, 32, 512, 0.05)
    vms = sg.arc_viewmats(rng, 8, radius=3.0, arc=2.0, jitter_deg=2.0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    geom = dict(means=t(sc.means), log_scales=t(sc.log_scales), quats=t(sc.quats),
                logit_opacity=t(sc.logit_opacity), rgb=t(sc.rgb))
    cam = CameraSpec(W, H, f, f, W / 2, H / 2)
    views = [View(t(v), cam) for v in vms]
    f512 = t(feat).to(torch.bfloat16)
    teacher, alphas = [], []
    for v in views:
        _, outs = render_features(geom, f512, v)
        teacher.append(outs[3].clone())
        alphas.append(outs[2].clone())
    return geom, views, teacher, alphas, f512, t(q)


def test_decoder_distillation_gain():
    from paper_2504_19409_amd.distill import Distiller, feature_errors, render_features
    geom, views, teacher, alphas, f512, q = _setup()
    train = [0, 1, 2, 4, 5, 7]
    held = [3, 6]
    d = Distiller(geom, [views[k] for k in train], [teacher[k] for k in train],
                  lr_latent=2e-2, lr_decoder=2e-3)
    y0, _ = d.decode(views[held[0]])
    e0 = feature_errors(y0, teacher[held[0]], alphas[held[0]], q)
    for it in range(600):
        d.step(it % len(train))
    torch.cuda.synchronize()
    errs = []
    for k in held:
        y, _ = d.decode(views[k])
        errs.append(feature_errors(y, teacher[k], alphas[k], q))
    print("\ninit", e0, "\nheld-out", errs, flush=True)
    for e in errs:
        assert e["rel_l2"] < 0.5 * e0["rel_l2"]
        # the teacher's per-Gaussian noise (0.05 per channel, norm ~1.1 against a unit
        # class vector) is beyond 16 latent channels; the class structure is not
        assert e["rel_l2"] <= 0.40, e
        assert e["argmax_agreement"] >= 0.97, e
    # speed: plain 512-channel render vs latent render + decode, same view
    v = views[held[0]]
    for _ in range(3):
        render_features(geom, f512, v)
        d.decode(v)
    torch.cuda.synchronize()
    n = 10
    t0 = time.perf_counter()
    for _ in range(n):
        render_features(geom, f512, v)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / n
    t0 = time.perf_counter()
    for _ in range(n):
        d.decode(v)
    torch.cuda.synchronize()
    t_dec = (time.perf_counter() - t0) / n
    print(f"plain 512-ch render {t_plain * 1e3:.3f} ms, latent render + decode {t_dec * 1e3:.3f} ms",
          flush=True)
    assert t_dec < t_plain
    # per-Gaussian feature storage: 16 vs 512 BF16 channels
    assert d.latent.shape[1] * 2 * 32 == f512.shape[1] * 2


def test_decoder_gain_full_scale():
    """The learned-decoder workload at full size: 500k Gaussians at 640x480,
    eight training and two held-out views on a 2 m arc, 800 training steps.
    On the held-out views the decoded map must halve the initial error and
    beat, by 10%, a render of every Gaussian's class-mean feature (what the
    class structure alone gives; the teacher's per-Gaussian noise is mostly
    beyond a 16-channel latent: measured 0.30-0.32 against 0.40-0.41 relative
    L2), keep the Eq. 12 labels of at least 97% of the covered pixels, render
    + decode faster than the plain 512-channel render, and store 32x fewer
    feature bytes per Gaussian."""
    from paper_2504_19409_amd.distill import decoder_experiment
    r = decoder_experiment()
    print("\n", r, flush=True)
    for e, c in zip(r["held"], r["class_mean"]):
        assert e["rel_l2"] < 0.5 * r["init"]["rel_l2"], e
        assert e["rel_l2"] <= 0.9 * c["rel_l2"], (e, c)
        assert e["argmax_agreement"] >= 0.97, e
    assert r["latent_render_decode_ms"] < r["plain_512_render_ms"]
    assert r["feature_bytes_per_gaussian"]["plain"] == 32 * r["feature_bytes_per_gaussian"]["latent"]
