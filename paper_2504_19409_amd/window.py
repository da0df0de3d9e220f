"""Keyframe-window mapping step: several views of one Gaussian set.

The paper maps over selected keyframes rather than every frame (Sec. 3.2).
One window step renders every view, forms each view's L1 upstream inside the
adjoint, and accumulates the Gaussian gradients over the views (the
library's `accumulate` mode) while every view keeps its own pose gradient.
All views' launches are recorded once into a HIP graph and replayed, so a
step costs one graph launch.  Each view owns its workspace; pair capacities
come from one eager sizing pass before capture; every view's status bits
are gathered on the device, and check() reads them (the mapping step does so
every few steps) so that a view that outgrew its capacity is reported rather
than silently rendered empty.
"""
from __future__ import annotations

import torch

from . import _capi
from .rasterizer import CameraSpec, Frame

GRAD_NAMES = ("means", "log_scales", "quats", "logit_opacity", "rgb", "feat")


class KeyframeWindow:
    def __init__(self, geom: dict, feat: torch.Tensor | None, views: list, targets: list,
                 weights=(0.5, 0.5, 0.0, 0.0), headroom: float = 1.1):
        """geom: means/log_scales/quats/logit_opacity/rgb device tensors;
        views: list of (viewmat [3,4] tensor, CameraSpec); targets: per view
        (t_rgb, t_depth, t_alpha, t_feat), None entries leave a group out;
        weights: of the colour, depth, opacity and feature L1 means (the
        default is Eq. 8's colour and depth terms at lambda_m = 0.5)."""
        self.geom, self.feat, self.views, self.targets = geom, feat, views, targets
        self.weights = weights
        self.headroom = headroom
        dev = geom["means"].device
        P = geom["means"].shape[1]
        C = 0 if feat is None else feat.shape[1]
        self._size_frames()
        shapes = dict(means=(3, P), log_scales=(3, P), quats=(4, P), logit_opacity=(P,),
                      rgb=(3, P), feat=(P, C))
        self.grads = {k: torch.zeros(shapes[k], device=dev) for k in GRAD_NAMES
                      if not (k == "feat" and C == 0)}
        self.pose = torch.zeros((len(views), 6), device=dev)
        self.loss = torch.zeros(1, device=dev)
        # status bits of every view's forward since the last check, OR-ed on
        # the device inside run() (so a captured step needs no host read)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.graph = None

    def _size_frames(self, scale: float = 1.0):
        """Pair capacity of every view from one eager sizing pass (at least
        ``scale`` times the previous capacity)."""
        old = getattr(self, "frames", None)
        self.frames = []
        for v, (vm, cam) in enumerate(self.views):
            fr = self._frame(vm, cam, None)
            fr.forward()
            flags, n = fr.read_status()
            if flags:
                fr = self._frame(vm, cam, n + 1024)
                fr.forward()
                flags, n = fr.read_status()
                assert flags == 0
            cap = int(n * self.headroom) + 4096
            if old is not None:
                cap = max(cap, int(old[v].max_pairs * scale))
            self.frames.append(self._frame(vm, cam, cap))
        self.outs = [fr.alloc_outputs() for fr in self.frames]

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
            torch.bitwise_or(self.status, fr.ws_view("status", torch.int32, 1), out=self.status)
            g = dict(self.grads)
            g["pose"] = self.pose[v]
            fr.backward_l1(self.outs[v], self.targets[v], self.weights, g, self.loss,
                           accumulate=True)

    def check(self):
        """Read (waits for the device) and clear the status bits the views
        raised since the last check; raise if a view overflowed its pair
        capacity (it rendered empty, so its gradients were wrong): call
        resize() and capture() again."""
        flags = int(self.status.item())
        self.status.zero_()
        if flags & _capi.FLAG_PAIR_OVERFLOW:
            raise RuntimeError("a keyframe view overflowed its pair capacity: the Gaussians "
                               "grew; call resize() (and capture() again)")
        return flags

    def resize(self, scale: float = 1.5):
        """New pair capacities for the current Gaussians and poses (at least
        ``scale`` times the old ones); drops a captured graph."""
        self._size_frames(scale)
        self.graph = None

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
