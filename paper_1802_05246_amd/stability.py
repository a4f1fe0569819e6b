"""Measured stability of the dissipative variants on the GPU.

The multi-dimensional dissipative method exists in two variants: the straightforward
one, with one interpolant per variable (Sec. 3.3, the "simple" method of Sec. 6.1),
and the one with the modified first step (Sec. 3.3, the "full" method).  Its Taylor
series in time either runs to the last non-zero stage (exact evolution of the cell
polynomials) or is truncated, as the paper's GPU kernels do with 2m+2 stages
(Sec. 6.1).  This module measures, through the library, how fast the worst mode
grows per full time step for each (variant, series, d, m, lambda = c dt / h).

Method: random coefficients on a small periodic grid, v = 0, advanced `steps` full
steps.  The scheme is translation invariant, so the per-coefficient means over the
nodes (the zero-wavenumber block, which holds the linearly growing mean-velocity
mode of the continuous problem) evolve on their own and are removed before taking
norms.  The fluctuation norm is sampled every `block` steps; nearly neutral modes make
it oscillate, so the growth per step compares the largest sample of the last third of
the run with the largest of the middle third: g = (max_last / max_middle)^(1/distance),
above 1 means an unstable mode.

Run:  python -m paper_1802_05246_amd.stability [--quick]
(one JSON line per case on stdout, a summary table on stderr)
"""
from __future__ import annotations

import argparse
import json
import math
import sys

from . import binding as B
from . import workloads as W

VARIANTS = {"full": W.DISS_FULL, "simple": W.DISS_SIMPLE}


def last_stage(series: str, m: int) -> int:
    """taylor_stages for a series label: "exact" (0: run to the last non-zero stage),
    "2m+1" or "2m+2" (the last stage computed; the paper's 2m+2 stages read as counting
    the s = 0 term gives 2m+1, read as stages 1..2m+2 gives 2m+2)."""
    return {"exact": 0, "2m+1": 2 * m + 1, "2m+2": 2 * m + 2}[series]


def fluctuation_norm(torch, u, w, tau):
    return math.sqrt(float(((u - u.mean(0)) ** 2).sum()) + tau * tau * float(((w - w.mean(0)) ** 2).sum()))


def window_growth(norms, block):
    """Growth per step from norms sampled every `block` steps (see the module docstring)."""
    k = len(norms) // 3
    mid, last = norms[k:2 * k], norms[2 * k:3 * k]
    if not all(map(math.isfinite, mid + last)) or max(mid) == 0.0:
        return float("inf")
    return (max(last) / max(mid)) ** (1.0 / (k * block))


def growth_per_step(d, m, lam, variant="full", series="exact", n=8, steps=400, block=10, seed=0,
                    precision=B.HW_FP64):
    """Growth factor per full step of the fluctuations (see the module docstring)."""
    import torch
    spec = W.make_spec(d, m, [n] * d, 0.0, 1.0, 1.0, cfl=lam, bc=W.PERIODIC,
                       method=VARIANTS[variant], taylor_stages=last_stage(series, m))
    u, v = W.random_state(spec, seed)
    v[:] = 0.0
    tau = 0.5 * spec.dt
    s = B.Solver(spec, precision=precision)
    norms = []
    try:
        s.set_state(u, v)
        B.hw_prepare_advance(s.h, block)
        for _ in range(steps // block):
            s.advance(block)
            norms.append(fluctuation_norm(torch, *s.get_state(), tau))
            if not math.isfinite(norms[-1]):
                break
    finally:
        s.close()
    return window_growth(norms, block)


def study(quick=False):
    """Yield one record per case: the largest growth over the grid sizes tried."""
    lams = [0.8, 1.0] if quick else [0.5, 0.8, 0.9, 0.95, 1.0]
    for d, ms, sizes in ((2, range(1, 7), (8, 16)), (3, range(1, 5), (4, 6))):
        for variant in ("full", "simple"):
            for series in ("exact", "2m+1", "2m+2"):
                for m in ms:
                    if quick and m not in (1, 3, 5):
                        continue
                    for lam in lams:
                        g = max(growth_per_step(d, m, lam, variant, series, n=n) for n in sizes)
                        yield {"d": d, "variant": variant, "series": series, "m": m, "lambda": lam,
                               "growth_minus_1": g - 1.0, "grids": list(sizes), "steps": 400}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--quick", action="store_true", help="fewer (m, lambda) points")
    args = ap.parse_args(argv)
    rows = []
    for rec in study(args.quick):
        print(json.dumps(rec), flush=True)
        rows.append(rec)
    print(f"{'d':>2} {'variant':>7} {'series':>6} {'m':>2} " + " ".join(
        f"lam={lam:<5}" for lam in sorted({r['lambda'] for r in rows})), file=sys.stderr)
    keys = sorted({(r["d"], r["variant"], r["series"], r["m"]) for r in rows},
                  key=lambda k: (k[0], k[1], ["exact", "2m+1", "2m+2"].index(k[2]), k[3]))
    for k in keys:
        vals = [r for r in rows if (r["d"], r["variant"], r["series"], r["m"]) == k]
        vals.sort(key=lambda r: r["lambda"])
        print(f"{k[0]:>2} {k[1]:>7} {k[2]:>6} {k[3]:>2} " + " ".join(
            f"{r['growth_minus_1']:+.1e}" for r in vals), file=sys.stderr)


if __name__ == "__main__":
    main()
