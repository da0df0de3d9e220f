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
