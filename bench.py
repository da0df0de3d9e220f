"""Throughput of one forward+backward render iteration of the feature-field
Gaussian rasterizer on one MI355X.

Workload (the tracking/mapping frame): 200,000 Gaussians drawn uniformly in
the camera frustum at 1-5 m, 640x480 pinhole camera (fx = fy = 525), RGB +
depth + accumulated opacity + 16-channel FP32 features, camera pose perturbed
by 1 cm / 1 degree from the pose the target images were rendered at.

One step = preprocess -> depth sort -> tile binning -> (tile sort -> tile
ranges, no-ops on this tile grid) -> compositing -> adjoint of the L1 loss
mean|rgb - t| + mean|depth - t| + mean|feat - t| (upstream formed inside the
compositing adjoint) -> preprocess adjoint + pose reduction, all in libgsff
kernels on one stream, inputs resident in HBM.

After the timed step, the same frame also times the other SLAM passes built
on the rasterizer, reported under config.slam: a tracking iteration (forward
without features, pose-only adjoint of the masked tracking loss, pose step),
the keyframe test's visibility record and co-visibility counts, the mapping
step's scale regulariser and fused Adam, and decode + query of the rendered
features against 20 labels.

Prints one JSON line (see the keys below); ``--gpus`` above 1 is refused: this
build runs on a single GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
# VALU issue peak from the unit counts: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# lane-instructions ("slots") per second = 78.6 TFLOP/s of non-packed FP32 FMA
# (packed FP32 is disabled on these machines).
VALU_PEAK_TSLOTS = 256 * 4 * 16 * 2.4e9 / 1e12
# LDS delivery peak: 256 bytes per clock per CU x 256 CUs x 2.4 GHz, in TB/s.
# The probe library measures it on the box (lane-delivered 16-byte reads at
# broadcast and per-lane addresses: about 146 and 119 TB/s), which rules out
# the 128 B/clk of the previous generation.
LDS_PEAK_TBS = 256 * 256 * 2.4e9 / 1e12
# LDS bytes a lane must receive per alpha evaluation: the Gaussian's image
# position, scaled conic and opacity (six floats).  The blending payload
# reaches the matrix cores once per wave and Gaussian, not per pixel.
LDS_BYTES_PER_EVAL = 24

# What the timed step computes in: the inputs, outputs and gradients are
# FP32; alpha, transmittance and every decision are FP32 VALU arithmetic; the
# blending sums (colour, depth, features) and the adjoint's per-tile
# contraction run on BF16 matrix cores with each FP32 operand split into a
# high and a low BF16 part (three products, FP32 accumulation: about 2^-16
# relative per product); depth keys and the pose sum are FP64.
DTYPE_LABEL = "f32 (blend sums: bf16x3 split MFMA, f32 accumulate)"
ARITHMETIC = ("FP32 alpha/transmittance/decisions; colour, depth and feature blend sums and "
              "the adjoint contraction as BF16 hi/lo split MFMA (hi*hi + lo*hi + hi*lo) with "
              "FP32 accumulation; FP64 depth keys and pose sum")

STAGES = ["preprocess", "sort_depth", "bin", "sort_tiles", "tile_ranges", "composite_fwd",
          "composite_bwd_l1", "preprocess_bwd"]
L1_WEIGHTS = (1.0, 1.0, 0.0, 1.0)  # rgb, depth, alpha, feature
# Stages that are a single kernel launch at this workload, whose event time is
# that kernel's launch duration; the roofline entry is for the longest of
# them.  The forward compositing kernel is the longest kernel of the step;
# the adjoint stage holds two launches (the L1 code pass, then the adjoint
# kernel), so its time is not one kernel's.
ONE_KERNEL_STAGES = ["composite_fwd"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="wall-clock budget of the CPU oracle sample")
    ap.add_argument("--no-graph", action="store_true", help="time eager launches only")
    ap.add_argument("--graph-steps", type=int, default=8,
                    help="whole steps captured in one graph (replayed back to back; each "
                         "step is the full forward + backward)")
    ap.add_argument("--workload", default="frame",
                    choices=["frame", "mixed", "decoder", "window"],
                    help="frame (default): 200k Gaussians, 640x480, 16-ch FP32; mixed: 1M "
                         "Gaussians, 1200x680, 64-ch BF16; decoder: 500k Gaussians, 640x480, "
                         "16-ch latent + learned decoder vs the plain 512-ch render; window: "
                         "8-view keyframe window, 1M Gaussians, 32-ch BF16, one graph")
    ap.add_argument("--profile-run", action="store_true",
                    help="for counter collection: eager steps only, no oracle work counts or "
                         "CPU baseline, plus one plain 256 MiB device copy whose counters "
                         "calibrate FETCH_SIZE / WRITE_SIZE, then a few decoder launches "
                         "(decode, decode + query, train step)")
    return ap.parse_args()


def build_problem(torch):
    from paper_2504_19409_amd import scenegen as sg
    from paper_2504_19409_amd.rasterizer import CameraSpec, Frame
    scene, _ = sg.workload_scene("frame")
    cam = scene.camera
    spec = CameraSpec(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    dev = dict(means=t(scene.means), log_scales=t(scene.log_scales), quats=t(scene.quats),
               logit_opacity=t(scene.logit_opacity), rgb=t(scene.rgb), feat=t(scene.feat))
    # targets: this library's render of the same scene at the unperturbed pose
    ident = t(sg.identity_viewmat())
    f0 = Frame(dev["means"], dev["log_scales"], dev["quats"], dev["logit_opacity"], dev["rgb"],
               dev["feat"], ident, spec)
    targets = [o.clone() for o in f0.forward()]
    # pair capacity from one sizing pass at the perturbed pose
    vm = t(cam.viewmat)
    f1 = Frame(dev["means"], dev["log_scales"], dev["quats"], dev["logit_opacity"], dev["rgb"],
               dev["feat"], vm, spec)
    f1.forward()
    flags, n = f1.read_status()
    assert flags == 0, "pair overflow while sizing"
    fr = Frame(dev["means"], dev["log_scales"], dev["quats"], dev["logit_opacity"], dev["rgb"],
               dev["feat"], vm, spec, max_pairs=int(n * 1.05) + 4096)
    return scene, fr, targets, n


class Step:
    """One forward+backward iteration issued stage by stage."""

    def __init__(self, torch, fr, targets):
        self.torch, self.fr = torch, fr
        self.targets = [targets[0], targets[1], None, targets[3]]  # alpha not in the loss
        self.outs = fr.alloc_outputs()
        self.loss = torch.zeros(1, device="cuda")
        self.grads = fr.make_grads()

    def run(self, events=None):
        fr = self.fr
        rec = (lambda i: events[i].record()) if events is not None else (lambda i: None)
        rec(0)
        fr.call_stage("gsff_preprocess")
        rec(1)
        fr.call_stage("gsff_sort_depth")
        rec(2)
        fr.call_stage("gsff_bin")
        rec(3)
        fr.call_stage("gsff_sort_tiles")
        rec(4)
        fr.call_stage("gsff_tile_ranges")
        rec(5)
        fr.composite_fwd(self.outs)
        rec(6)
        # the L1 code pass also builds the work items and clears the loss and
        # the feature gradient (accumulate = 0)
        fr.composite_bwd_l1(self.outs, self.targets, L1_WEIGHTS, self.grads, self.loss)
        rec(7)
        fr.preprocess_bwd(self.grads)
        rec(8)


def tracking_rate(torch, fr, targets, K, warmup):
    """Tracking iterations per second on the same frame, from its perturbed
    pose toward the targets: forward without features, the pose-only adjoint
    of the masked tracking loss (Eq. 6) and the pose step, replayed from a HIP
    graph (the captured step keeps one Adam step count; timing only)."""
    from paper_2504_19409_amd.tracking import pose_adam_step, pose_state, tracking_masks
    st = fr.settings
    keep_feat = st.render_features
    vm = fr.tensors[-1]
    keep_vm = vm.clone()
    st.render_features = 0
    try:
        rgb, depth, alpha, _ = fr.alloc_outputs()
        outs = (rgb, depth, alpha, None)
        fr.forward(outs=outs)
        # edge threshold: keeps about 30% of this frame's pixels
        mv, me = tracking_masks(targets[0], alpha, 0.0025, 0.5)
        dev = rgb.device
        d_pose, state = torch.zeros(6, device=dev), pose_state(dev)
        delta, loss = torch.zeros(6, device=dev), torch.zeros(1, device=dev)

        def iteration(step):
            fr.forward(outs=outs)
            fr.backward_tracking(outs, targets[0], targets[1], mv, me, 0.9, d_pose, loss)
            pose_adam_step(vm, d_pose, state, step, 1e-3, 3e-3, delta=delta)

        for k in range(1, warmup + 1):
            iteration(k)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            iteration(warmup + 1)
        torch.cuda.current_stream().wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            iteration(warmup + 2)
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(K):
            g.replay()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / K * 1e3
        assert fr.read_status()[0] == 0, "pair overflow while tracking"
        return {"it_per_s": round(1e3 / ms, 1), "ms_per_iter": round(ms, 4),
                "features": "off", "lambda_t": 0.9,
                "edge_mask_kept": int(me.sum()), "vis_mask_kept": int(mv.sum()),
                "timing": "graph replay"}
    finally:
        st.render_features = keep_feat
        vm.copy_(keep_vm)


def keyframe_rates(torch, fr, K):
    """Durations of the keyframe test's two passes on the frame (Sec. 3.2,
    Eq. 5): the visibility record of the last forward and the co-visibility
    counts of two records, from HIP events around K launches of each."""
    from paper_2504_19409_amd import _capi
    from paper_2504_19409_amd.rasterizer import _ptr, _stream
    from paper_2504_19409_amd.tracking import covisibility
    fr.forward()
    vis = torch.empty(fr.P, dtype=torch.uint8, device="cuda")
    other = fr.visibility(0.5).clone()
    counts = torch.empty(2, dtype=torch.int32, device="cuda")
    L = _capi.load()

    def timed(fn):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(K):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / K * 1e3

    t_vis = timed(lambda: fr.visibility(0.5, out=vis))
    t_cov = timed(lambda: L.gsff_covisibility(_ptr(vis), _ptr(other), fr.P, _ptr(counts),
                                              _stream()))
    both, either = covisibility(vis, other)
    return {"visibility_us": round(t_vis, 1), "covisibility_us": round(t_cov, 1),
            "visible": int(vis.sum()), "iou_same_pose": round(both / max(either, 1), 4)}


def mapping_rates(torch, fr, K):
    """Durations of the mapping step's two passes beyond the window's
    forward + adjoint (Sec. 3.2, Eqs. 7-8) on the frame's Gaussians: the scale
    regulariser and the fused Adam step over all six parameter groups, from
    HIP events around K launches (on copies: the frame's Gaussians stay)."""
    from paper_2504_19409_amd.mapping import adam_step, scale_reg, scale_reg_workspace
    means, log_scales, quats, logit, rgb, feat, _ = fr.tensors
    params = [x.clone() for x in (means, log_scales, quats, logit, rgb, feat)]
    grads = [torch.randn_like(x) * 1e-3 for x in params]
    groups = [(p, g, torch.zeros_like(p), torch.zeros_like(p), 1e-3)
              for p, g in zip(params, grads)]
    ws = scale_reg_workspace(fr.P)
    loss = torch.zeros(1, device="cuda")

    def timed(fn):
        fn(1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for k in range(K):
            fn(k + 2)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / K * 1e3

    t_reg = timed(lambda k: scale_reg(params[1], 0.01, grads[1], loss, True, ws))
    t_adam = timed(lambda k: adam_step(groups, k))
    n = sum(p.numel() for p in params)
    return {"scale_reg_us": round(t_reg, 1), "adam_us": round(t_adam, 1), "adam_elements": n,
            "adam_gbs": round(n * 28 / (t_adam * 1e-6) / 1e9, 1)}


def query_rates(torch, fr, K):
    """Decode + query (Eqs. 10, 12) of the frame's rendered features (BF16)
    against 20 query vectors, beside the plain decode to the 512-channel map,
    from HIP events around K launches of each."""
    from paper_2504_19409_amd import decoder as dec
    outs = fr.forward(out_feat_dtype=torch.bfloat16)
    X = outs[3].reshape(16, -1)
    n = X.shape[1]
    params = dec.init_params(0)
    g = torch.Generator(device="cpu").manual_seed(1)
    Q = (torch.randn(20, 512, generator=g) / 20).cuda()
    ws_dec = dec.workspace(n)

    def timed(fn):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(K):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / K * 1e3

    t_query = timed(lambda: dec.query(X, params, Q))
    Y = torch.empty((512, n), dtype=torch.bfloat16, device="cuda")
    t_dec = timed(lambda: dec.forward(X, params, ws_dec, out=Y))
    T = (torch.randn(512, n, generator=g) * 0.5).to(torch.bfloat16).cuda()
    loss = torch.zeros(1, device="cuda")
    t_train = timed(lambda: dec.train_step(X, params, T, ws_dec, None, loss))
    map_bytes = 512 * n * 2
    return {"queries": 20, "pixels": n, "decode_query_us": round(t_query, 1),
            "decode_512_map_us": round(t_dec, 1),
            "decode_512_map_gbs": round(map_bytes / (t_dec * 1e-6) / 1e9, 1),
            "decoder_train_step_us": round(t_train, 1)}


def algorithmic_work(scene, n_pairs, torch):
    """Per-stage algorithmic bytes (HBM) and the compositing evaluation counts
    from the oracle's exact work counts (pairs with support, alpha
    evaluations up to each pixel's stop, contributing pairs)."""
    import oracle
    oracle.build(force=False)
    p, c = oracle.scene_dicts(scene)
    wc = oracle.work_counts(p, c, 16)
    P, C = scene.P, scene.C
    HW = scene.camera.width * scene.camera.height
    return wc, dict(P=P, C=C, HW=HW, n_pairs=n_pairs)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def walked_pairs(torch, fr):
    """(tile, Gaussian) pairs the last forward walked (the adjoint's rows)."""
    lay = fr.layout
    nt = lay.tiles_x * lay.tiles_y
    rg = fr.ws_view("tile_list_ranges", torch.int32, 2 * nt).view(nt, 2).cpu()
    return int((rg[:, 1] - rg[:, 0]).sum())


def cpu_baseline(scene, budget_s):
    """The FP64 oracle (single-threaded C++) on whole frames of the same
    workload: forward + backward with an L1-shaped upstream, repeated until the
    time budget is spent, with this process pinned to one host core."""
    import oracle
    from paper_2504_19409_amd import scenegen as sg
    oracle.build(force=False)
    p, c = oracle.scene_dicts(scene)
    rng = np.random.default_rng(0)
    W, H, C = scene.camera.width, scene.camera.height, scene.C
    gr, gd, ga, gf = sg.upstream_signs(rng, W, H, C)
    g = dict(g_rgb=gr, g_depth=gd, g_alpha=ga, g_feat=gf)
    allowed = sorted(os.sched_getaffinity(0))
    core = allowed[-1]
    os.sched_setaffinity(0, {core})
    try:
        n = 0
        t0 = time.perf_counter()
        while True:
            oracle.render(p, c)
            oracle.backward(p, c, g)
            n += 1
            el = time.perf_counter() - t0
            if el >= budget_s:
                break
    finally:
        os.sched_setaffinity(0, set(allowed))
    return dict(value=n / el, unit="it/s", cores=1, kind="oracle",
                sample=f"{n} full 640x480 / 200k-Gaussian / 16-ch frames, forward + backward, "
                       f"FP64 single-threaded C++ oracle pinned to core {core}, {el:.1f} s",
                host_cores=os.cpu_count(), host_cores_allowed=len(allowed),
                cpu_model=_cpu_model())


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(2)
    if args.workload != "frame":
        out = {"mixed": bench_mixed, "decoder": bench_decoder,
               "window": bench_window}[args.workload](torch, args)
        print(json.dumps(out), flush=True)
        return
    scene, fr, targets, n_pairs = build_problem(torch)
    step = Step(torch, fr, targets)
    log(f"pairs {n_pairs}, workspace {fr.ws_bytes / 1e6:.1f} MB")
    if args.profile_run:
        # counter calibration: two plain streaming kernels of known size, an
        # elementwise add (256 MiB read + 256 MiB written) and the runtime's
        # buffer copy (the same)
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.add(src, 1.0, out=dst)
        dst.copy_(src)
        for _ in range(args.steps):
            step.run()
        torch.cuda.synchronize()
        # the decoder kernels of the query leg: decode, decode + query, train step
        query_rates(torch, fr, 2)
        torch.cuda.synchronize()
        log("profile run done")
        return
    for _ in range(args.warmup):
        step.run()
    torch.cuda.synchronize()

    # eager, with per-stage events
    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(STAGES) + 1)]
          for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        step.run(ev[k])
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t0) / K * 1e3
    stage_ms = {s: float(np.median([ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(K)]))
                for i, s in enumerate(STAGES)}
    log("eager ms/step %.4f" % eager_ms)
    for s in STAGES:
        log(f"  {s:16s} {stage_ms[s] * 1e3:9.1f} us")

    # the same step replayed from a HIP graph (launch overhead removed)
    graph_ms, graph_dist = None, None
    if not args.no_graph:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            step.run()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        ref = [g.clone() for g in step.grads.values()]
        # steps per graph (the launch of a graph is paid once per S): the
        # largest divisor of K not above --graph-steps, so exactly K are timed
        S = max(1, min(args.graph_steps, K))
        while K % S:
            S -= 1
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(S):
                step.run()
        torch.cuda.synchronize()
        for _ in range(3):
            g.replay()
        torch.cuda.synchronize()
        for a, b in zip(step.grads.values(), ref):
            d = (a - b).norm() / max(b.norm(), 1e-30)
            assert float(d) < 1e-4, "graph replay differs from eager"
        for _ in range((args.warmup + S - 1) // S):
            g.replay()
        torch.cuda.synchronize()
        # per-replay events (median, p10, p90 of a replay's time per step)
        # inside the wall-clock bracket; K steps = R replays of S
        R = K // S
        gev = [torch.cuda.Event(enable_timing=True) for _ in range(R + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gev[0].record()
        for k in range(R):
            g.replay()
            gev[k + 1].record()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - t0) / (R * S) * 1e3
        per = np.array([gev[k].elapsed_time(gev[k + 1]) / S for k in range(R)])
        graph_dist = {"median_ms": round(float(np.median(per)), 4),
                      "p10_ms": round(float(np.percentile(per, 10)), 4),
                      "p90_ms": round(float(np.percentile(per, 90)), 4)}
        log("graph ms/step %.4f (median %.4f, p10 %.4f, p90 %.4f)"
            % (graph_ms, graph_dist["median_ms"], graph_dist["p10_ms"], graph_dist["p90_ms"]))

    ms = min(eager_ms, graph_ms) if graph_ms else eager_ms
    value = 1e3 / ms

    # the other SLAM passes on the same frame (Sec. 3.2): tracking iteration,
    # keyframe test, mapping step's regulariser and optimiser
    slam = {"tracking": tracking_rate(torch, fr, targets, K, args.warmup),
            "keyframe": keyframe_rates(torch, fr, K), "mapping": mapping_rates(torch, fr, K),
            "query": query_rates(torch, fr, K)}
    log("tracking iteration %.4f ms; visibility %.1f us, covisibility %.1f us; scale reg %.1f "
        "us, adam %.1f us" % (slam["tracking"]["ms_per_iter"], slam["keyframe"]["visibility_us"],
                              slam["keyframe"]["covisibility_us"],
                              slam["mapping"]["scale_reg_us"], slam["mapping"]["adam_us"]))
    log("decode + query %.1f us (decode to the 512-channel map %.1f us)"
        % (slam["query"]["decode_query_us"], slam["query"]["decode_512_map_us"]))

    wc, sizes = algorithmic_work(scene, n_pairs, torch)
    wc["walked"] = walked_pairs(torch, fr)
    try:
        from paper_2504_19409_amd import probe
        peaks = probe.measure()
    except Exception as e:  # the probe library is a measurement aid only
        log(f"probe unavailable: {e}")
        peaks = {}
    log(f"measured peaks {peaks}")
    dom = max(ONE_KERNEL_STAGES, key=lambda s: stage_ms[s])
    roof = roofline_for(dom, stage_ms[dom], wc, sizes, peaks)
    bound_us = {s: round(stage_bound_us(s, wc, sizes), 2) for s in STAGES}
    step_bound = sum(bound_us.values())
    out = {
        "metric": "fwd+bwd render iterations/sec at 640x480, 200k Gaussians, 16-ch features",
        "value": round(value, 2), "unit": "it/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE_LABEL, "data": "synthetic",
        "config": {"workload": "tracking/mapping frame: 200k Gaussians, 640x480, fx=fy=525, "
                               "RGB+depth+alpha+16-ch FP32 features, pose perturbed 1 cm/1 deg",
                   "gaussians": scene.P, "width": 640, "height": 480, "channels": 16,
                   "arithmetic": ARITHMETIC,
                   "timing": (f"graph replay ({S} steps per graph)" if graph_ms and graph_ms < eager_ms
                              else "eager"),
                   "eager_ms": round(eager_ms, 4),
                   "graph_ms": round(graph_ms, 4) if graph_ms else None,
                   "graph_replay_dist": graph_dist,
                   "stage_us": {s: round(v * 1e3, 1) for s, v in stage_ms.items()},
                   "pairs": n_pairs, "work": wc, "slam": slam,
                   "stage_bound_us": bound_us,
                   "step_roofline": {"bound_us": round(step_bound, 2),
                                     "frac": round(step_bound / (ms * 1e3), 4),
                                     "note": "sum over stages of the time at each stage's "
                                             "limiting roofline, over the measured step"},
                   "peaks_measured": peaks},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scene, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def _line(metric, value, unit, K, W, ms, config, roofline=None, dtype=DTYPE_LABEL):
    return {"metric": metric, "value": round(value, 3), "unit": unit, "n_gpus": 1, "steps": K,
            "warmup": W, "ms_per_step": round(ms, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
            "config": config, "roofline": roofline, "cpu_baseline": None}


def _replay_ms(torch, run, K, warmup):
    """Capture run() into a graph and time K replays (wall clock inside
    synchronisations, plus per-replay events for the median)."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(K):
        g.replay()
        ev[k + 1].record()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / K * 1e3
    per = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(K)])
    return ms, {"median_ms": round(float(np.median(per)), 4),
                "p10_ms": round(float(np.percentile(per, 10)), 4),
                "p90_ms": round(float(np.percentile(per, 90)), 4)}


def bench_mixed(torch, args):
    """Mixed-precision frame: 1M Gaussians, 1200x680, fx = fy = 600, 64-channel
    BF16 payload with FP32 compositing; targets rendered at the scene pose,
    the step at a pose perturbed by 1 cm / 1 degree; one step = the frame
    step (forward + fused-L1 adjoint + preprocess adjoint with the pose)."""
    from paper_2504_19409_amd import scenegen as sg
    from paper_2504_19409_amd.rasterizer import CameraSpec, Frame
    scene, _ = sg.workload_scene("mixed")
    cam = scene.camera
    spec = CameraSpec(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    d = dict(means=t(scene.means), log_scales=t(scene.log_scales), quats=t(scene.quats),
             logit_opacity=t(scene.logit_opacity), rgb=t(scene.rgb),
             feat=t(scene.feat).to(torch.bfloat16))
    mk = lambda vm, mp=None: Frame(d["means"], d["log_scales"], d["quats"], d["logit_opacity"],
                                   d["rgb"], d["feat"], vm, spec, max_pairs=mp)
    f0 = mk(t(cam.viewmat))
    targets = [o.clone() for o in f0.forward()]
    prng = np.random.default_rng(1003)
    vm, _ = sg.perturbed_viewmat(prng, cam.viewmat, 0.01, 1.0)
    vmt = t(np.ascontiguousarray(vm, np.float32))
    f1 = mk(vmt)
    f1.forward()
    flags, n = f1.read_status()
    assert flags == 0, "pair overflow while sizing"
    fr = mk(vmt, int(n * 1.05) + 4096)
    del f0, f1
    step = Step(torch, fr, targets)
    for _ in range(args.warmup):
        step.run()
    torch.cuda.synchronize()
    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(STAGES) + 1)]
          for _ in range(K)]
    for k in range(K):
        step.run(ev[k])
    torch.cuda.synchronize()
    stage_ms = {s: float(np.median([ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(K)]))
                for i, s in enumerate(STAGES)}
    ms, dist = _replay_ms(torch, step.run, K, args.warmup)
    assert fr.read_status()[0] == 0
    log("mixed: graph ms/step %.4f; stages %s" % (ms, {k: round(v * 1e3, 1)
                                                        for k, v in stage_ms.items()}))
    cfg = {"workload": "mixed-precision frame: 1M Gaussians, 1200x680, fx=fy=600, RGB+depth+"
                       "alpha+64-ch BF16 features, FP32 compositing, pose perturbed 1 cm/1 deg",
           "gaussians": scene.P, "width": cam.width, "height": cam.height, "channels": 64,
           "payload": "bf16", "timing": "graph replay", "graph_replay_dist": dist,
           "stage_us": {k: round(v * 1e3, 1) for k, v in stage_ms.items()}, "pairs": n}
    return _line("fwd+bwd render iterations/sec at 1200x680, 1M Gaussians, 64-ch BF16 features",
                 1e3 / ms, "it/s", K, args.warmup, ms, cfg)


def bench_decoder(torch, args):
    """Learned decoder: 500k Gaussians at 640x480 with 512-channel class-
    structured BF16 features; the decoded frame (16-ch latent render + the
    1x1 MLP to 512 channels) against the plain 512-channel render, after
    training on eight views of a 2 m arc (two held out)."""
    from paper_2504_19409_amd.distill import decoder_experiment
    r = decoder_experiment(steps=800)
    ms = r["latent_render_decode_ms"]
    n_px = r["width"] * r["height"]
    map_bytes = 512 * n_px * 2
    dec_s = r["decode_ms"] * 1e-3
    roof = {"bound": "hbm", "achieved": round(map_bytes / dec_s / 1e9, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(map_bytes / dec_s / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": None, "stage": "decoder_forward",
            "other_bound": {"bound": "mfma", "unit": "TFLOP/s", "peak": 2500.0,
                            "achieved": round(2 * n_px * (16 * 128 + 128 * 512) / dec_s / 1e12,
                                              1),
                            "frac": round(2 * n_px * (16 * 128 + 128 * 512) / dec_s / 2.5e15,
                                          4)}}
    log("decoder: %s" % r)
    cfg = {"workload": "learned decoder: 500k Gaussians, 640x480, 16-ch BF16 latent render + 1x1 "
                       "MLP 16-128-512 (BF16 MFMA, FP32 accumulation) vs the plain 512-ch BF16 "
                       "render", "result": r}
    return _line("decoded 512-ch feature frames/sec at 640x480, 500k Gaussians", 1e3 / ms,
                 "frames/s", 10, 2, ms, cfg, roof, dtype="bf16 (FP32 accumulation)")


def bench_window(torch, args):
    """Keyframe window: 1M Gaussians with 32-ch BF16 features, 8 views
    alternating 640x480 (fx 525) and 1200x680 (fx 600) on a 2 m arc; one step =
    every view's forward and fused-L1 adjoint with the Gaussian gradients
    accumulated over the views, replayed from one graph."""
    from paper_2504_19409_amd import scenegen as sg
    from paper_2504_19409_amd.rasterizer import CameraSpec
    from paper_2504_19409_amd.window import KeyframeWindow
    rng = np.random.default_rng(5)
    P, C = 1_000_000, 32
    sc = sg.make_scene(P, 640, 480, 525.0, 525.0, 320.0, 240.0, C, seed=5, rng=rng)
    vms = sg.arc_viewmats(rng, 8, radius=3.0, arc=2.0, jitter_deg=2.0)
    sizes = [(640, 480, 525.0), (1200, 680, 600.0)] * 4
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    geom = dict(means=t(sc.means), log_scales=t(sc.log_scales), quats=t(sc.quats),
                logit_opacity=t(sc.logit_opacity), rgb=t(sc.rgb))
    feat = t(sc.feat).to(torch.bfloat16)
    views = [(t(vm), CameraSpec(W, H, f, f, W / 2, H / 2)) for (W, H, f), vm in zip(sizes, vms)]
    targets = []
    for (vm, cam) in views:
        g = torch.Generator(device="cpu").manual_seed(len(targets))
        targets.append([torch.rand((3, cam.height, cam.width), generator=g).cuda(),
                        (1 + 4 * torch.rand((cam.height, cam.width), generator=g)).cuda(), None,
                        torch.randn((C, cam.height, cam.width), generator=g).cuda()])
    win = KeyframeWindow(geom, feat, views, targets, weights=(1.0, 1.0, 0.0, 1.0))
    win.run()
    win.check()
    K = max(args.steps // 10, 10)
    ms, dist = _replay_ms(torch, win.run, K, 3)
    assert win.check() == 0
    log("window: graph ms/step %.3f" % ms)
    cfg = {"workload": "keyframe window: 1M Gaussians, 32-ch BF16 features, 8 views alternating "
                       "640x480 (fx 525) and 1200x680 (fx 600) on a 2 m arc, fwd + fused-L1 "
                       "adjoint of every view, gradients accumulated, one graph",
           "gaussians": P, "views": 8, "channels": C, "timing": "graph replay",
           "graph_replay_dist": dist}
    return _line("keyframe-window steps/sec (8 views fwd+bwd, 1M Gaussians, 32-ch BF16)",
                 1e3 / ms, "steps/s", K, 3, ms, cfg)


# Measured HBM traffic of the dominant kernel, from the rocprofv3 counter
# summary committed beside the kernel profiles.  It is used only while the
# kernel source still hashes to the value recorded with the counters.
TRAFFIC_PROFILE = {
    "composite_fwd": os.path.join(ROOT, "profiles", "composite_fwd_640x480_200k_traffic.md"),
    "composite_bwd_l1": os.path.join(ROOT, "profiles", "composite_bwd_640x480_200k_traffic.md"),
}
KERNEL_SOURCE = os.path.join(ROOT, "paper_2504_19409_amd", "csrc", "composite.hip")


def measured_traffic(stage):
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE[stage]).read()
        src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in text.splitlines()
                  if line.startswith(("source_sha256:", "traffic_bytes_per_launch:")))
    if fields.get("source_sha256", "").strip() != src:
        return None  # the kernel changed since the counters were taken
    try:
        return int(fields["traffic_bytes_per_launch"].strip())
    except (KeyError, ValueError):
        return None


def _alu_slots(stage, wc):
    """Vector-ALU lane slots of a compositing kernel (a transcendental, issued
    at quarter rate, counts 4): alpha evaluation (per pixel and Gaussian walked
    up to the pixel's stop) 15; forward, per contributing pair (transmittance,
    stop test, weight, hi / lo split) 8; adjoint, per contributing pair
    (transmittance recovery, weight, g . c, dL/dalpha, suffix sum, dL/dpower)
    16.  The colour, depth, feature and per-Gaussian sums run on the matrix
    cores and are not counted."""
    per_contrib = 8 if stage == "composite_fwd" else 16
    return wc["evals"] * 15 + wc["contribs"] * per_contrib


def stage_bound_us(stage, wc, sz):
    """Time of a stage at its limiting roofline (nominal peaks), microseconds,
    from its algorithmic work: HBM bytes for the streaming stages, the larger
    of vector-ALU slots and LDS lane bytes for the compositing kernels (plus
    the upstream pass's HBM bytes for the adjoint)."""
    P, C, HW, M = sz["P"], sz["C"], sz["HW"], sz["n_pairs"]
    hbm = lambda b: b / (HBM_PEAK_GBS * 1e9) * 1e6
    if stage in ("composite_fwd", "composite_bwd_l1"):
        t_alu = _alu_slots(stage, wc) / (VALU_PEAK_TSLOTS * 1e12) * 1e6
        t_lds = wc["tile_evals"] * LDS_BYTES_PER_EVAL / (LDS_PEAK_TBS * 1e12) * 1e6
        t = max(t_alu, t_lds)
        if stage == "composite_bwd_l1":  # outputs and targets read once, codes written
            t += hbm(HW * (2 * (5 + C)) * 4 + HW * (1 + (C + 15) // 16) * 4)
        return t
    return hbm(algorithmic_bytes(stage, sz, wc))


def algorithmic_bytes(stage, sz, wc):
    P, C, HW, M = sz["P"], sz["C"], sz["HW"], sz["n_pairs"]
    return {
        "preprocess": P * (44 + 12) + P * (48 + 8 + 8),
        # a stable sort of P 4-byte keys with 4-byte ids: one read and one
        # write of both per 8-bit pass
        "sort_depth": 4 * P * 8 * 2,
        # keys read, super-tile entries (id + mask) written once
        "bin": P * 8 * 2 + M * 6,
        "sort_tiles": 0,
        "tile_ranges": 0,
        # adjoint rows (one per walked pair, 10 + C floats) read once,
        # parameters read, gradients written
        "preprocess_bwd": wc.get("walked", 0) * (10 + C) * 4 + P * (44 + 12) + P * (56 + 4 * C),
    }[stage]


def roofline_for(stage, ms, wc, sz, peaks=None):
    """Roofline entry of the dominant stage: algorithmic work per launch over the
    measured average launch time.  Work per unit is stated in the design notes.

    The compositing kernels have two candidate bounds; the limiting one is the
    one whose time at peak is longer: vector-ALU issue (``_alu_slots``) and
    LDS lane delivery (LDS_BYTES_PER_EVAL per lockstep evaluation of the
    tile).  ``peaks`` (measured on the box by the probe library) are reported
    beside the nominal ones."""
    peaks = peaks or {}
    sec = ms * 1e-3
    if stage in ("composite_fwd", "composite_bwd_l1"):
        slots = _alu_slots(stage, wc)
        lds_bytes = wc["tile_evals"] * LDS_BYTES_PER_EVAL
        alu = slots / sec / 1e12
        lds = lds_bytes / sec / 1e12
        t_lds, t_alu = lds_bytes / (LDS_PEAK_TBS * 1e12), slots / (VALU_PEAK_TSLOTS * 1e12)
        traffic = measured_traffic(stage)
        other = {"bound": "alu", "achieved": round(alu, 3), "peak": round(VALU_PEAK_TSLOTS, 2),
                 "unit": "Tslot/s", "frac": round(alu / VALU_PEAK_TSLOTS, 4),
                 "work": int(slots)}
        main_ = {"bound": "lds", "achieved": round(lds, 3), "peak": round(LDS_PEAK_TBS, 2),
                 "unit": "TB/s", "frac": round(lds / LDS_PEAK_TBS, 4), "work": int(lds_bytes)}
        if "lds_broadcast_tbs" in peaks:
            main_["peak_measured"] = peaks["lds_broadcast_tbs"]
            main_["frac_measured"] = round(lds / peaks["lds_broadcast_tbs"], 4)
        if t_alu > t_lds:
            main_, other = other, main_
        out = dict(main_)
        out.update({"traffic": traffic, "stage": stage, "other_bound": other})
        return out
    bytes_ = algorithmic_bytes(stage, sz, wc)
    achieved = bytes_ / sec / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "stage": stage}
    if "hbm_read_gbs" in peaks:
        out["peak_measured"] = peaks["hbm_read_gbs"]
    return out


if __name__ == "__main__":
    main()
