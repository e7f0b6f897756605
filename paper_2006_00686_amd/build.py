"""Build libxrt.so (gfx950) in-tree with hipcc.

    python -m paper_2006_00686_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libxrt.so")
BUILD = os.path.join(HERE, "_build")

SOURCES = ["xrt_plan.cpp", "xrt_project.hip", "xrt_gather.hip", "xrt_vec.hip", "xrt_conv.hip", "xrt_batch.cpp", "xrt_csr.hip",
           "xrt_simplex.hip"]

# Packed FP32 instructions are switched off for all device code; float atomics map to
# the hardware instructions; no NaN is ever formed in the kernels (infinities are), so
# min/max need no signalling-NaN quieting.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics", "-fno-honor-nans", "-mno-amdgpu-ieee", "-Wall", "-Wno-unused-result",
             "-I" + os.path.join(HERE, "..", "include")]


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"]
        cmd = [_hipcc()] + lang + HIP_FLAGS + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
