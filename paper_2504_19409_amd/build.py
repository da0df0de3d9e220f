"""Build libgsff.so (HIP, gfx950) in-tree with hipcc.

Every translation unit is compiled for gfx950 only, with packed-FP32 VALU
instructions disabled, then linked into ``paper_2504_19409_amd/libgsff.so``.
The same sources compiled with ``-DGSFF_CHECKED=1`` make the checked build
``libgsff_checked.so`` (every data-dependent index tested against its buffer,
failures recorded in the workspace status word instead of faulting), and
``probe.hip`` the roofline microbenchmarks ``libgsff_probe.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgsff.so")
PROBE_LIB = os.path.join(HERE, "libgsff_probe.so")
CHECKED_LIB = os.path.join(HERE, "libgsff_checked.so")
CHECKED_BUILD = os.path.join(BUILD, "checked")
SOURCES = ["capi.hip", "preprocess.hip", "sort.hip", "composite.hip", "decoder.hip",
           "tracking.hip", "mapping.hip", "f64.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def common_flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-Wno-unused-result",
            "-I", os.path.join(HERE, "..", "include")]


def _compile(src: str, checked: bool = False) -> str:
    out = CHECKED_BUILD if checked else BUILD
    obj = os.path.join(out, os.path.splitext(os.path.basename(src))[0] + ".o")
    cmd = [hipcc(), *common_flags(), *(["-DGSFF_CHECKED=1"] if checked else []), "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}{' (checked)' if checked else ''}:\n{r.stderr}")
    return obj


def _link(lib: str, objs) -> None:
    tmp = lib + ".tmp"
    r = subprocess.run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)


def build(verbose: bool = False) -> str:
    os.makedirs(CHECKED_BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = [(s, False) for s in srcs] + [(s, True) for s in srcs] + [("probe.hip", False)]
    # the largest translation units first, so the pool drains evenly
    jobs.sort(key=lambda j: -os.path.getsize(os.path.join(CSRC, j[0])))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        objs = dict(zip(jobs, ex.map(lambda j: _compile(*j), jobs)))
    _link(LIB, [objs[(s, False)] for s in srcs])
    _link(CHECKED_LIB, [objs[(s, True)] for s in srcs])
    _link(PROBE_LIB, [objs[("probe.hip", False)]])
    if verbose:
        print("built", LIB, CHECKED_LIB, "and", PROBE_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
