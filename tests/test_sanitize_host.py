"""Address and undefined-behaviour sanitizer runs of the host code, on the
CPU: the oracle's C core (tests/sanitize/oracle_driver.c) and the library's
host-only planners, workspace queries and argument checks
(tests/sanitize/host_driver.cpp).  The library's host-logic sources are
compiled with the sanitizers on their host side only; the kernel sources
link from the regular build.  No device is touched."""
import glob
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1805_11775_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr)
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_core_under_sanitizers():
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-fsanitize=address,undefined",
          "-fno-omit-frame-pointer", os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "hos_oracle.c"), "-lm", "-o", exe])
    r = _run([exe], env=dict(ENV, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1"))
    assert "oracle driver: ok" in r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC) or shutil.which("g++") is None,
                    reason="hipcc or g++ not available")
def test_host_planners_under_sanitizers():
    from paper_1805_11775_amd import build as b
    kernels = sorted(glob.glob(os.path.join(b.BUILD_DIR, "k_*.hip.o")))
    srcs = sorted(glob.glob(os.path.join(CSRC, "k_*.hip")))
    if len(kernels) != len(srcs) or any(
            os.path.getmtime(o) < os.path.getmtime(s) for o, s in zip(kernels, srcs)):
        b.build()
        kernels = sorted(glob.glob(os.path.join(b.BUILD_DIR, "k_*.hip.o")))
    os.makedirs(OUT, exist_ok=True)
    host_srcs = sorted(glob.glob(os.path.join(CSRC, "hos_*.hip")))

    def compile_one(src):
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        # the sanitizers on the host side only (the device code is left alone)
        _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC,
              "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-omit-frame-pointer",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Wno-unused-value", "-Wno-unused-command-line-argument", "-c", src, "-o", obj])
        return obj

    with ThreadPoolExecutor(max_workers=min(8, len(host_srcs))) as ex:
        objs = list(ex.map(compile_one, host_srcs))
    drv = os.path.join(OUT, "host_driver.o")
    _run(["g++", "-O1", "-g", "-std=c++17", "-I", os.path.join(ROOT, "include"),
          "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-c",
          os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"), "-o", drv])
    exe = os.path.join(OUT, "host_driver")
    _run(["g++", "-fsanitize=address,undefined", drv, *objs, *kernels, "-L/opt/rocm/lib",
          "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    r = _run([exe], env=ENV)
    assert "host driver: ok" in r.stdout
