"""Build the gfx950 shared library libhj.so in-tree with hipcc.

The library has a plain C interface (include/hj.h); the Python binding loads
it with ctypes.  Kernel instantiations are split over several translation
units that compile in parallel.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libhj.so")
BUILD = os.path.join(HERE, "_build")

SOURCES = (["hj_api.hip"] + [f"hj_inst_{t}_{i}.hip" for t in ("f64", "f32") for i in range(5)]
           + [f"hj_inst_c64_{i}.hip" for i in range(4)] + [f"hj_inst_r64_{i}.hip" for i in range(3)]
           + ["hj_inst_paper.hip"])

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + INCLUDE, "-I" + CSRC,
]


# The FP64 descent kernels run one wave per SIMD whatever their register use
# (65536 one-lane tasks fill the device once), so their instruction schedule
# is built for instruction-level parallelism rather than occupancy, with the
# target's own register-pressure trackers (n=10 solve 177 -> 166 ms measured).
ILP_FLAGS = ["-mllvm", "-amdgpu-sched-strategy=max-ilp", "-mllvm", "-amdgpu-use-amdgpu-trackers=1"]
PER_SOURCE = {src: ILP_FLAGS for src in
              [f"hj_inst_f64_{i}.hip" for i in range(4)] + [f"hj_inst_c64_{i}.hip" for i in range(3)]
              + [f"hj_inst_r64_{i}.hip" for i in range(3)]}


def _compile(src: str, extra=()) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *PER_SOURCE.get(src, []), *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    subprocess.check_call(cmd)
    return obj


def build(verbose: bool = False, resource_usage: bool = False) -> str:
    """Compile every HIP source and link libhj.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    extra = ["-Rpass-analysis=kernel-resource-usage"] if resource_usage else []
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, extra), SOURCES))
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, resource_usage="--resources" in sys.argv)
