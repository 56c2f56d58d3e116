"""Build libspasm.so (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libspasm.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "api.hip", "serve.hip", "noalloc.hip")]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 (v_pk_*_f32) code generation
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # device code only: no NaN operands are expected, so min/max need no NaN quieting and
    # fuse with DPP lane moves; the host keeps IEEE NaN semantics for input validation
    "-Xarch_device", "-fno-honor-nans",
    # instruction scheduling for latency rather than occupancy: the stage-2 kernels run at
    # a fixed occupancy set by their launch bounds (measured: 10-block tower launch -2.1 %,
    # 4-block -1.2 %, the same results)
    "-mllvm", "-amdgpu-sched-strategy=max-ilp",
    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False, extra=()) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *FLAGS, *extra, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
