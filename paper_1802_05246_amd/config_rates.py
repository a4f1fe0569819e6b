"""Rates of the library on every workload recipe: the 1-D standing waves (64 cells,
m = 3), the 2-D dissipative pulses (512^2, m = 3), the 2-D conservative standing wave
(2048^2 Dirichlet, m = 4, c dt = h), the 3-D dissipative pulses (256^3, m = 3) and the
batch of 256 independent 2-D problems, in FP64 and FP32, each advanced through
hw_advance / hw_batch_advance (one captured hipGraph per run) on data resident in HBM.

Per workload: cell-updates/s (one output node of one half step), and the algorithmic
flop and byte rates from the per-cell-update counts of the survey's counting rules
(read one node and write one node per dissipative cell-update; read the other grid's
node, the old node and write the new one per conservative cell-update).

Run:  python -m paper_1802_05246_amd.config_rates [--only c2,c3] [--copy-calibration]
(one JSON line per (workload, precision) on stdout, a table on stderr; --copy-calibration
first runs a plain copy of 2^28 float32 values three times, the reference kernel that
scales the FETCH_SIZE / WRITE_SIZE counters of a profiling pass)
"""
from __future__ import annotations

import argparse
import json
import sys
import time

from . import binding as B
from . import workloads as W

# algorithmic flops per cell-update (survey counting rules); None: not tabulated
FLOPS = {"c1": 286, "c2": 4464, "c3": 4932, "c4": 48272, "c5": None}


def _values_per_update(spec):
    """Values moved per cell-update at the boundary of one half step."""
    nu = (spec.m + 1) ** spec.d
    if spec.method == W.CONSERVATIVE:
        return 3 * nu
    return 2 * (nu + max(spec.m, 1) ** spec.d)


def _cells_per_step(spec):
    return spec.nodes(W.PRIMAL) + spec.nodes(W.DUAL)


def _start(s, works):
    for i, w in enumerate(works):
        kw = {"i": i} if s.batch else {}
        if w.spec.method == W.CONSERVATIVE:
            if w.u_half is not None:
                s.set_state(w.u0, w.u_half, **kw)
            else:
                s.cons_startup(w.u0, None, **kw)
        else:
            s.set_state(w.u0, w.v0, **kw)


def measure(torch, name, works, precision, steps):
    batch = len(works) > 1 or name == "c5"
    s = (B.Solver(problems=[w.spec for w in works], precision=precision) if batch
         else B.Solver(works[0].spec, precision=precision))
    try:
        _start(s, works)
        B.hw_prepare_advance(s.h, steps)
        s.advance(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.advance(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    finally:
        s.close()
    cells = sum(_cells_per_step(w.spec) for w in works) * steps
    elem = 8 if precision == B.HW_FP64 else 4
    moved = sum(_cells_per_step(w.spec) * _values_per_update(w.spec) for w in works) * steps * elem
    rec = {"workload": name, "precision": "fp64" if precision == B.HW_FP64 else "fp32",
           "problems": len(works), "steps": steps, "seconds": el,
           "cell_updates_per_s": cells / el, "algorithmic_gbs": moved / el / 1e9}
    if FLOPS[name] is not None:
        rec["algorithmic_tflops"] = FLOPS[name] * cells / el / 1e12
    return rec


def workloads(name, device):
    if name == "c1":
        return [W.c1_1d()], None
    if name == "c2":
        return [W.c2_2d()], 20
    if name == "c3":
        return [W.c3_2d()], 10
    if name == "c4":
        return [W.c4_3d(device=device)], 20
    return W.c5_batch(), 4


def copy_calibration(torch, elems=1 << 28):
    """A plain elementwise copy of `elems` float32 values, three times (each reads 4 B and
    writes 4 B per element)."""
    a = torch.ones(elems, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()


def main(argv=None):
    import torch
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--only", default="c1,c2,c3,c4,c5", help="comma-separated workloads")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run the counter-calibration copy before the workloads")
    args = ap.parse_args(argv)
    if args.copy_calibration:
        copy_calibration(torch)
    rows = []
    for name in args.only.split(","):
        works, steps = workloads(name, "cuda")
        if steps is None:
            steps = works[0].steps
        for prec in (B.HW_FP64, B.HW_FP32):
            rec = measure(torch, name, works, prec, steps)
            print(json.dumps(rec), flush=True)
            rows.append(rec)
    print(f"{'workload':8} {'prec':5} {'cell-updates/s':>15} {'GB/s (alg.)':>12} {'TFLOP/s (alg.)':>15}",
          file=sys.stderr)
    for r in rows:
        tf = r.get("algorithmic_tflops")
        print(f"{r['workload']:8} {r['precision']:5} {r['cell_updates_per_s']:15.3e} "
              f"{r['algorithmic_gbs']:12.1f} {'' if tf is None else f'{tf:15.2f}'}", file=sys.stderr)


if __name__ == "__main__":
    main()
