"""Keyframe-window mapping step: several views of one Gaussian set.

The paper maps over selected keyframes rather than every frame (Sec. 3.2).
One window step renders every view, forms each view's L1 upstream inside the
adjoint, and accumulates the Gaussian gradients over the views (the
library's `accumulate` mode) while every view keeps its own pose gradient.
All views' launches are recorded once into a HIP graph and replayed, so a
step costs one graph launch.  Each view owns its workspace; pair capacities
come from one eager sizing pass before capture.
"""
from __future__ import annotations

import torch

from .rasterizer import CameraSpec, Frame

GRAD_NAMES = ("means", "log_scales", "quats", "logit_opacity", "rgb", "feat")


class KeyframeWindow:
    def __init__(self, geom: dict, feat: torch.Tensor | None, views: list, targets: list,
                 weights=(1.0, 1.0, 0.0, 1.0), headroom: float = 1.1):
        """geom: means/log_scales/quats/logit_opacity/rgb device tensors;
        views: list of (viewmat [3,4] tensor, CameraSpec); targets: per view
        (t_rgb, t_depth, t_alpha, t_feat), None entries leave a group out."""
        self.geom, self.feat, self.views, self.targets = geom, feat, views, targets
        self.weights = weights
        dev = geom["means"].device
        P = geom["means"].shape[1]
        C = 0 if feat is None else feat.shape[1]
        # sizing pass: pair capacity of every view
        self.frames = []
        for vm, cam in views:
            fr = self._frame(vm, cam, None)
            fr.forward()
            flags, n = fr.read_status()
            if flags:
                fr = self._frame(vm, cam, n + 1024)
                fr.forward()
                flags, n = fr.read_status()
                assert flags == 0
            self.frames.append(self._frame(vm, cam, int(n * headroom) + 4096))
        self.outs = [fr.alloc_outputs() for fr in self.frames]
        shapes = dict(means=(3, P), log_scales=(3, P), quats=(4, P), logit_opacity=(P,),
                      rgb=(3, P), feat=(P, C))
        self.grads = {k: torch.zeros(shapes[k], device=dev) for k in GRAD_NAMES
                      if not (k == "feat" and C == 0)}
        self.pose = torch.zeros((len(views), 6), device=dev)
        self.loss = torch.zeros(1, device=dev)
        self.graph = None

    def _frame(self, vm, cam: CameraSpec, max_pairs):
        g = self.geom
        return Frame(g["means"], g["log_scales"], g["quats"], g["logit_opacity"], g["rgb"],
                     self.feat, vm, cam, max_pairs=max_pairs)

    def run(self):
        """One window step, eager."""
        for t in self.grads.values():
            t.zero_()
        self.pose.zero_()
        self.loss.zero_()
        for v, fr in enumerate(self.frames):
            fr.forward(outs=self.outs[v])
            g = dict(self.grads)
            g["pose"] = self.pose[v]
            fr.backward_l1(self.outs[v], self.targets[v], self.weights, g, self.loss,
                           accumulate=True)

    def capture(self):
        """Record run() into a HIP graph (after one eager warm-up on a side
        stream, as graph capture requires)."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.run()
        return self.graph

    def replay(self):
        self.graph.replay()
