"""Distilling the 512-channel feature field into 16-channel latents plus the
learned 1x1 decoder (the lift o(.) of Eq. 11).

Teacher: the plain rasterizer rendering every Gaussian's 512-channel BF16
feature (eight 64-channel passes).  Student: a 16-channel BF16 latent per
Gaussian, rendered by the same rasterizer and decoded by the BF16-MFMA MLP.
Training runs entirely in this library's kernels -- latent render, fused
decoder L1 step, feature-only rasterizer backward -- with PyTorch's Adam
updating the FP32 master copies.  The geometry is frozen (the paper optimises
the feature field after the geometry, Sec. 3.3).
"""
from __future__ import annotations

import dataclasses

import torch

from . import decoder as dec
from .rasterizer import CameraSpec, Frame


@dataclasses.dataclass
class View:
    viewmat: torch.Tensor   # [3, 4] float32 device
    cam: CameraSpec


def render_features(geom: dict, feat: torch.Tensor, view: View, max_pairs=None):
    """Forward render; returns (frame, outputs) with a BF16 feature map."""
    fr = Frame(geom["means"], geom["log_scales"], geom["quats"], geom["logit_opacity"],
               geom["rgb"], feat, view.viewmat, view.cam, max_pairs=max_pairs)
    outs = fr.forward(out_feat_dtype=torch.bfloat16)
    return fr, outs


class Distiller:
    def __init__(self, geom: dict, views: list, teacher: list, latent_seed: int = 0,
                 lr_latent: float = 1e-2, lr_decoder: float = 1e-3, max_pairs=None):
        self.geom, self.views, self.teacher = geom, views, teacher
        P = geom["means"].shape[1]
        g = torch.Generator(device="cpu").manual_seed(latent_seed)
        self.latent = (0.1 * torch.randn(P, dec.LATENT, generator=g)).cuda().requires_grad_(True)
        self.params = {k: v.requires_grad_(True) for k, v in dec.init_params(latent_seed).items()}
        self.opt = torch.optim.Adam([
            {"params": [self.latent], "lr": lr_latent},
            {"params": list(self.params.values()), "lr": lr_decoder}])
        H, W = views[0].cam.height, views[0].cam.width
        self.ws = dec.workspace(H * W)
        self.max_pairs = max_pairs
        self.loss = torch.zeros(1, device="cuda")

    def step(self, k: int) -> None:
        view = self.views[k]
        lat16 = self.latent.detach().to(torch.bfloat16)
        fr, outs = render_features(self.geom, lat16, view, self.max_pairs)
        X = outs[3].reshape(dec.LATENT, -1)
        g = dec.train_step(X, {n: p.detach() for n, p in self.params.items()},
                           self.teacher[k].reshape(dec.OUT, -1), self.ws, loss=self.loss)
        grads = {"feat": torch.empty_like(self.latent)}
        fr.backward(None, None, None, g["dX"], grads)  # feature-only adjoint
        self.latent.grad = grads["feat"]
        for n in ("W1", "b1", "W2", "b2"):
            self.params[n].grad = g["d" + n]
        self.opt.step()

    def decode(self, view: View, out_dtype=torch.bfloat16):
        lat16 = self.latent.detach().to(torch.bfloat16)
        fr, outs = render_features(self.geom, lat16, view, self.max_pairs)
        X = outs[3].reshape(dec.LATENT, -1)
        Y = dec.forward(X, {n: p.detach() for n, p in self.params.items()}, self.ws, out_dtype)
        return Y, outs


def feature_errors(Y: torch.Tensor, T: torch.Tensor, alpha: torch.Tensor, queries: torch.Tensor):
    """Relative L1 / L2 of a decoded map against the teacher on covered pixels
    (alpha > 0.5), and the agreement of argmax_l f(x) q(l) (Eq. 12's label
    rule) between the two maps."""
    m = (alpha.reshape(-1) > 0.5)
    y = Y.reshape(Y.shape[0], -1)[:, m].float()
    t = T.reshape(T.shape[0], -1)[:, m].float()
    rel_l1 = float((y - t).abs().sum() / t.abs().sum())
    rel_l2 = float((y - t).norm() / t.norm())
    ly = (queries @ y).argmax(0)
    lt = (queries @ t).argmax(0)
    agree = float((ly == lt).float().mean())
    return dict(rel_l1=rel_l1, rel_l2=rel_l2, argmax_agreement=agree, pixels=int(m.sum()))


def _time_ms(fn, n=10, warm=2):
    for _ in range(warm):
        fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(n):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / n


def decoder_experiment(P: int = 500_000, W: int = 640, H: int = 480, f: float = 525.0,
                       n_views: int = 10, held=(3, 7), steps: int = 800, seed: int = 4,
                       lr_latent: float = 2e-2, lr_decoder: float = 2e-3, timing: bool = True):
    """The learned-decoder workload (Sec. 3.3, Eq. 11): P Gaussians with
    class-structured 512-channel BF16 features (32 classes), n_views cameras on
    a 2 m arc, the plain 512-channel render of every view as the teacher,
    16-channel latents + decoder trained on the views not in ``held`` and
    judged on the held-out ones.  Returns a dict: the held-out errors
    (relative L1 / L2 on covered pixels, Eq. 12 argmax agreement), the same
    errors of a render with every Gaussian carrying its class's mean feature
    (what the class structure alone gives: the teacher's per-Gaussian noise is
    beyond the latent), per-frame times of the plain render and of latent
    render + decode, the train step time, and the feature bytes per Gaussian."""
    import numpy as np

    from . import scenegen as sg
    rng = np.random.default_rng(seed)
    sc = sg.make_scene(P, W, H, f, f, W / 2, H / 2, 0, seed=seed, rng=rng)
    feat, labels, q = sg.semantic_features(rng, sc.means, 32, 512, 0.05)
    vms = sg.arc_viewmats(rng, n_views, radius=3.0, arc=2.0, jitter_deg=2.0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    geom = dict(means=t(sc.means), log_scales=t(sc.log_scales), quats=t(sc.quats),
                logit_opacity=t(sc.logit_opacity), rgb=t(sc.rgb))
    cam = CameraSpec(W, H, f, f, W / 2, H / 2)
    views = [View(t(v), cam) for v in vms]
    f512 = t(feat).to(torch.bfloat16)
    # class-mean features: what a representation of the classes alone renders
    cls = np.zeros((32, 512))
    np.add.at(cls, labels, feat.astype(np.float64))
    cls /= np.maximum(np.bincount(labels, minlength=32), 1)[:, None]
    fcls = t(cls[labels].astype(np.float32)).to(torch.bfloat16)
    del feat
    qt = t(q)
    teacher, alphas = [], []
    for v in views:
        _, outs = render_features(geom, f512, v)
        teacher.append(outs[3].clone())
        alphas.append(outs[2].clone())
    train = [k for k in range(n_views) if k not in held]
    d = Distiller(geom, [views[k] for k in train], [teacher[k] for k in train],
                  lr_latent=lr_latent, lr_decoder=lr_decoder)
    y0, _ = d.decode(views[held[0]])
    init = feature_errors(y0, teacher[held[0]], alphas[held[0]], qt)
    for it in range(steps):
        d.step(it % len(train))
    torch.cuda.synchronize()
    out = dict(P=P, width=W, height=H, views=n_views, held_out=list(held), steps=steps,
               init=init, held=[], class_mean=[])
    for k in held:
        y, _ = d.decode(views[k])
        out["held"].append(feature_errors(y, teacher[k], alphas[k], qt))
        _, oc = render_features(geom, fcls, views[k])
        out["class_mean"].append(feature_errors(oc[3], teacher[k], alphas[k], qt))
    out["feature_bytes_per_gaussian"] = dict(plain=512 * 2, latent=dec.LATENT * 2)
    if timing:
        v = views[held[0]]
        out["plain_512_render_ms"] = round(_time_ms(lambda: render_features(geom, f512, v)), 4)
        out["latent_render_decode_ms"] = round(_time_ms(lambda: d.decode(v)), 4)
        lat16 = d.latent.detach().to(torch.bfloat16)
        _, outs = render_features(geom, lat16, v)
        X = outs[3].reshape(dec.LATENT, -1)
        pr = {n: p.detach() for n, p in d.params.items()}
        Y = torch.empty((dec.OUT, W * H), dtype=torch.bfloat16, device="cuda")
        out["decode_ms"] = round(_time_ms(lambda: dec.forward(X, pr, d.ws, out=Y)), 4)
        tg = teacher[held[0]].reshape(dec.OUT, -1)
        out["train_step_ms"] = round(_time_ms(lambda: dec.train_step(X, pr, tg, d.ws)), 4)
        out["distill_step_ms"] = round(_time_ms(lambda: d.step(0), n=5), 4)
    return out
