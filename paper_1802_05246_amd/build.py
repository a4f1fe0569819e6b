"""Build libhermite_wave.so (HIP, gfx950) in-tree with hipcc.

The library is the C ABI declared in include/hermite_wave.h; every half step runs
in its kernels.  The Hermite tables are regenerated from exact rationals first.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhermite_wave.so")
SOURCES = ["api.cpp", "cellmap.cpp", "tune.cpp", "kernels_generic.hip", "kernel_tiled3d.hip", "kernel_dense.hip",
           "kernel_cmap3d.hip", "probes.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # keep the compiler from forming packed FP32 (v_pk_*_f32) instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_tables.py")],
                          stdout=subprocess.DEVNULL)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", CSRC, "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
