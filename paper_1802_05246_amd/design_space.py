"""Rates of the kernel forms on the 3-D dissipative m = 3 workload (256^3 periodic cube,
8 Gaussian pulses, c dt / h = 0.9): the composed-map MFMA kernel (exact and cut series),
the fused tiled MFMA kernel (exact series), the
fused generic kernel with the exact series and with the series cut after stage 2m+1
or 2m+2 (the paper's GPU kernels ran 2m+2 stages, Sec. 6.1), and the two-kernel form
(interpolants written to memory by one kernel and read back by a second, the paper's
two-kernel design of Sec. 6.1), in FP32 and FP64.

Run:  python -m paper_1802_05246_amd.design_space [--n 256] [--steps 3]
(one JSON line per form on stdout)
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import time

from . import binding as B
from . import workloads as W

FORMS = [("composed map on the matrix cores, exact series", B.HW_KERNEL_COMPOSED, 0),
         ("composed map, series cut after stage 2m+2", B.HW_KERNEL_COMPOSED, 8),
         ("tiled fused, exact series", B.HW_KERNEL_TILED, 0),
         ("generic fused, exact series", B.HW_KERNEL_GENERIC, 0),
         ("generic fused, series cut after stage 2m+1", B.HW_KERNEL_GENERIC, 7),
         ("generic fused, series cut after stage 2m+2", B.HW_KERNEL_GENERIC, 8),
         ("two kernels (interpolants through memory), exact series", B.HW_KERNEL_SPLIT, 0)]


def measure(torch, w, precision, kernel, stages, steps):
    spec = dataclasses.replace(w.spec, taylor_stages=stages)
    s = B.Solver(spec, precision=precision, kernel=kernel)
    try:
        s.set_state(w.u0, w.v0)
        B.hw_prepare_advance(s.h, steps)
        B.hw_advance(s.h, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.hw_advance(s.h, steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    finally:
        s.close()
        torch.cuda.empty_cache()
    return 2 * spec.nodes(W.PRIMAL) * steps / el, el / (2 * steps)


def main(argv=None):
    import torch
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--steps", type=int, default=3)
    args = ap.parse_args(argv)
    B.lib()
    w = W.c4_3d(n=args.n, device="cuda")
    for pname, prec in (("fp32", B.HW_FP32), ("fp64", B.HW_FP64)):
        for name, kernel, stages in FORMS:
            rate, per = measure(torch, w, prec, kernel, stages, args.steps)
            print(json.dumps({"form": name, "precision": pname, "n": args.n, "steps": args.steps,
                              "cell_updates_per_s": rate, "ms_per_half_step": per * 1e3}), flush=True)


if __name__ == "__main__":
    main()
