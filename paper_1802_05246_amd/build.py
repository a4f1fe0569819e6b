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
           "kernel_cmap3d.hip", "kernel_cmap2d.hip", "probes.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # keep the compiler from forming packed FP32 (v_pk_*_f32) instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]
OBJDIR = os.path.join(HERE, "_build")


def build(verbose: bool = False) -> str:
    """Compile every source to an object in _build/ (in parallel), then link the library."""
    from concurrent.futures import ThreadPoolExecutor
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_tables.py")],
                          stdout=subprocess.DEVNULL)
    os.makedirs(OBJDIR, exist_ok=True)
    objs = [os.path.join(OBJDIR, s + ".o") for s in SOURCES]

    def compile_one(i):
        cmd = [HIPCC, *FLAGS, "-I", CSRC, "-c", "-o", objs[i], os.path.join(CSRC, SOURCES[i])]
        if verbose:
            print(" ".join(cmd), flush=True)
        return subprocess.run(cmd).returncode

    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        codes = list(ex.map(compile_one, range(len(SOURCES))))
    bad = [SOURCES[i] for i, c in enumerate(codes) if c != 0]
    if bad:
        raise subprocess.CalledProcessError(1, "hipcc " + " ".join(bad))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-fPIC", "-shared", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
