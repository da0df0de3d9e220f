"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

* the oracle (oracle/gsff_oracle.cpp), built with g++ and the sanitizers into
  the driver tests/sanitize/oracle_check.cpp, which calls every entry point
  on small seeded scenes and on the degenerate ones (no Gaussians, all
  culled, non-finite and zero parameters, a 1x1 image, no channels);
* the C ABI's host side (csrc/capi.hip, the sanitizers on the host pass
  only) linked with the library's other objects, driven by
  tests/sanitize/capi_check.cpp over a grid of workspace sizes (valid and
  unrepresentable) and the argument validation of every entry point -- all
  paths that return before anything is launched, so no GPU is needed.

Any sanitizer report aborts the driver (-fno-sanitize-recover=all).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2504_19409_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("g++"):
        pytest.skip("no g++")
    exe = str(tmp_path / "oracle_check")
    _run(["g++", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fno-omit-frame-pointer",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          os.path.join(SAN, "oracle_check.cpp"), os.path.join(ROOT, "oracle", "gsff_oracle.cpp"),
          "-o", exe])
    r = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert "all entry points ok" in r.stdout


def test_capi_host_side_under_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("no ROCm compilers")
    from paper_2504_19409_amd import build
    objs = [os.path.join(build.BUILD, s.replace(".hip", ".o")) for s in build.SOURCES
            if s != "capi.hip"]
    if not all(os.path.exists(o) for o in objs):
        build.build()
    capi_o = str(tmp_path / "capi.o")
    _run([HIPCC, *build.common_flags(), "-O1", "-g",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-Xarch_host", "-fno-sanitize-recover=all",
          "-c", os.path.join(CSRC, "capi.hip"), "-o", capi_o])
    lib = str(tmp_path / "libgsff_san.so")
    _run([HIPCC, f"--offload-arch={build.ARCH}", "-shared", "-fPIC",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-o", lib, capi_o, *objs])
    exe = str(tmp_path / "capi_check")
    _run([CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"),
          os.path.join(SAN, "capi_check.cpp"), f"-L{tmp_path}", "-lgsff_san",
          f"-Wl,-rpath,{tmp_path}", "-o", exe])
    # the HIP runtime the library links is not instrumented: no leak check
    r = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert "host sanitizer run: ok" in r.stdout
