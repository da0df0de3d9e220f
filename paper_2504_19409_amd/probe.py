"""Measured roofline denominators on the current GPU (libgsff_probe.so):
LDS read delivery per lane (distinct and broadcast addresses) and HBM
streaming read bandwidth, each timed with events on the current stream."""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
PROBE_PATH = os.path.join(_HERE, "libgsff_probe.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(PROBE_PATH):
            raise RuntimeError(f"{PROBE_PATH} is not built; run paper_2504_19409_amd/build.py")
        L = ctypes.CDLL(PROBE_PATH)
        L.gsff_probe_lds.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_void_p]
        L.gsff_probe_hbm_read.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                          ctypes.c_void_p, ctypes.c_void_p]
        _lib = L
    return _lib


def _timed(fn, reps=5):
    fn()
    best = None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    return best


def lds_tbs(broadcast: bool, blocks_per_cu=8, steps=2000, cus=256) -> float:
    """Lane-delivered LDS read bandwidth, TB/s (best of five launches)."""
    L = _load()
    blocks = cus * blocks_per_cu
    sink = torch.empty(blocks * 256, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ms = _timed(lambda: L.gsff_probe_lds(int(broadcast), blocks, steps,
                                          ctypes.c_void_p(sink.data_ptr()), s))
    return blocks * 256 * steps * 16 * 16 / (ms * 1e-3) / 1e12


def hbm_read_gbs(nbytes=1 << 30, blocks=4096) -> float:
    """Streaming read bandwidth from HBM, GB/s (best of five launches)."""
    L = _load()
    src = torch.empty(nbytes // 4, device="cuda").fill_(1.0)
    sink = torch.empty(blocks * 256, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    n16 = nbytes // 16
    ms = _timed(lambda: L.gsff_probe_hbm_read(ctypes.c_void_p(src.data_ptr()), n16, blocks,
                                               ctypes.c_void_p(sink.data_ptr()), s))
    return nbytes / (ms * 1e-3) / 1e9


def measure() -> dict:
    return {"lds_broadcast_tbs": round(lds_tbs(True), 1),
            "lds_per_lane_tbs": round(lds_tbs(False), 1),
            "hbm_read_gbs": round(hbm_read_gbs(), 1)}


if __name__ == "__main__":
    print(measure())
