"""Build librewl.so (HIP kernels + host runtime) for gfx950 with hipcc.

Flags: -ffp-contract=off keeps every floating-point expression a sequence of
single IEEE operations (no fused multiply-add), -packed-fp32-ops off keeps the
compiler from forming packed FP32 instructions, and the instruction-level-
parallelism scheduling strategy orders each basic block for latency rather
than register pressure: the sweep runs one wave per SIMD, so occupancy gains
nothing and the in-order wave's stalls are what cost time.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librewl.so")
SOURCES = ["rewl_kernels.hip", "rewl_api.cpp"]


def hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(verbose=False):
    """Compile every source every time it is called (no staleness check)."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-mllvm", "-amdgpu-sched-strategy=max-ilp",
           "-Wall", "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", tmp]
    cmd += [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
