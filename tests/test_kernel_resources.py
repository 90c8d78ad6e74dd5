"""The matrix-core contractions must not spill to scratch memory: each runs
one wave per SIMD with its accumulators filling the register file, so a
spill (which the compiler introduces silently when a change adds a few live
values) costs 10-20 % of the kernel.  Compiles the sources for gfx950 with
the resource-usage remarks and checks every contraction kernel."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1805_11775_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _usage(src):
    cmd = [HIPCC, "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "--cuda-device-only", "-c", os.path.join(CSRC, src), "-o", os.devnull,
           "-Rpass-analysis=kernel-resource-usage"]
    out = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr[-2000:]
    kernels, cur = {}, None
    for line in out.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and cur:
            kernels[cur] = int(m.group(1))
    return kernels


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.parametrize("src,pattern", [
    ("k_c3.hip", r"k_c3_contract|k_c3_items"),
    ("k_c4.hip", r"k_c4_contract|k_c5_contract"),
    ("k_adjoint.hip", r"k_adj_contract"),
])
def test_contractions_do_not_spill(src, pattern):
    usage = _usage(src)
    hits = {k: v for k, v in usage.items() if re.search(pattern, k)}
    assert hits, "no kernel matched %s in %s" % (pattern, src)
    spilled = {k: v for k, v in hits.items() if v}
    assert not spilled, spilled
