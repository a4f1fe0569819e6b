"""Benchmark: cell-updates/s of the 3-D dissipative Hermite method, m = 3, on the
256^3 periodic unit cube with 8 Gaussian pulses (lambda = c dt/h = 0.9), FP32 form
against the FP64 form (and the BF16-operand form), with the L2 error reached.

One step = one full time step = two half steps over all 256^3 cells (two
cell-updates per node).  The timed region is `hw_advance(K)`: a hipGraph of 2K
half-step kernel launches on the current stream, inputs resident in HBM.

Prints ONE JSON line (rank 0, N = 1).  Only one GPU is used; --gpus N > 1 exits.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s, 3-D m=3, at stated L2 error; FP32-MFMA vs FP64 form"
HBM_PEAK_GBS = 8000.0
PEAKS_TFLOPS = {"fp32": 157.3, "fp64": 78.6, "bf16": 2500.0}
# algorithmic work of one cell-update of the 3-D dissipative full method, m = 3:
# flops of the interpolants (centre rows of p0, q0, the three mixed interpolants),
# the modified first-step Laplacian and the closed-form time sums, counted per cell
# without sharing between neighbouring cells; bytes = read one node + write one node
FLOPS_PER_CELL = 48272
BYTES_PER_CELL = {"fp32": 2 * 91 * 4, "fp64": 2 * 91 * 8}
# work the composed-map kernel executes per cell-update: 184 products of 16x16x4 (1024
# multiply-adds) per 16 cells, i.e. 11 776 multiply-adds on the matrix cores (padded class
# rows included), plus 1 460 vector additions of the corner butterflies
EXECUTED_FLOPS_PER_CELL = 2 * 11776 + 1460
# matrix-core busy fraction of the same kernel from its counters (SQ_BUSY_CYCLES /
# SQ_VALU_MFMA_BUSY_CYCLES pass), tied to the source it was measured on like the traffic
MFMA_BUSY_RECORD = {
    "source_sha256": "c24eced0708b2188e9e287d4ea0e7c271b541b19c1ab5ddf97d7f121387893c0",
    "busy_frac": 0.50,
    "profile": "profiles/k_cmap3d-diss3d_m3_256cube-sq_counters.md",
}


# HBM traffic of one launch of the dominant kernel (the FP32 composed-map half step on this
# workload), from two rocprofv3 --pmc passes (FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch), each scaled by the ratio of true to counted bytes of a plain copy of
# known size measured in the same pass (the --copy-calibration leg).  The record is
# tied to the source it was measured on: after any change of that file the traffic
# is reported as null until the counters are taken again.
TRAFFIC_RECORD = {
    "source_sha256": "c24eced0708b2188e9e287d4ea0e7c271b541b19c1ab5ddf97d7f121387893c0",
    "fetch_bytes": 8931630032,  # FETCH_SIZE 4361270.3 KiB x 1048576/524302.8 (copy: 1 GiB read)
    "write_bytes": 6174015488,  # WRITE_SIZE 6029312.0 KiB x 1048576/1048576.0 (copy: 1 GiB written)
    "profile": "profiles/k_cmap3d-diss3d_m3_256cube-hbm_bytes.md",
}
# the kernel's source files (the kernel and its device helpers); the digest is over their
# contents in this order
TRAFFIC_SOURCE = [os.path.join(ROOT, "paper_1802_05246_amd", "csrc", f) for f in ("kernel_cmap3d.hip", "buffer_io.h")]
COPY_ELEMS = 1 << 28  # float32 elements of the calibration copy (1 GiB read + 1 GiB written)


def source_digest(paths=TRAFFIC_SOURCE):
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_bytes():
    rec = TRAFFIC_RECORD
    if not rec or rec.get("source_sha256") != source_digest():
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def mfma_busy():
    rec = MFMA_BUSY_RECORD
    if not rec or rec.get("source_sha256") != source_digest():
        return None
    return rec["busy_frac"]


def copy_calibration(torch):
    """A plain elementwise copy of COPY_ELEMS float32 values (reads 4 B and writes 4 B
    per element): the reference kernel for scaling the FETCH_SIZE / WRITE_SIZE
    counters of a profiling pass."""
    a = torch.ones(COPY_ELEMS, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--fp64-steps", type=int, default=None,
                    help="timed steps of the FP64 form (default: same as --steps)")
    ap.add_argument("--kernel", choices=["auto", "composed", "tiled", "generic"], default="auto")
    ap.add_argument("--no-tiled", action="store_true",
                    help="skip the tiled-kernel FP32 form reported beside")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-error", action="store_true")
    ap.add_argument("--no-bf16", action="store_true", help="skip the BF16-operand form")
    ap.add_argument("--cpu-layers", type=int, default=40,
                    help="z-layers of the grid in the oracle's timed sample")
    ap.add_argument("--cpu-layers-1t", type=int, default=3,
                    help="z-layers of the oracle's single-thread sample")
    ap.add_argument("--accuracy-steps", type=int, default=200,
                    help="steps of the untimed accuracy leg (the workload's length); 0: skip")
    ap.add_argument("--no-probes", action="store_true", help="skip the measured-peak probes")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run the plain copy used to scale HBM byte counters")
    return ap.parse_args()


def timed_advance(torch, B, solver_h, steps, warmup):
    """warmup steps, then exactly `steps` steps bracketed by synchronisation and HIP
    events on the launch stream; returns (elapsed s, event ms)."""
    stream = torch.cuda.current_stream()
    if warmup:
        B.hw_advance(solver_h, warmup, stream.cuda_stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    B.hw_advance(solver_h, steps, stream.cuda_stream)
    e1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return t1 - t0, e0.elapsed_time(e1)


def run_form(torch, B, W, w, precision, kernel, steps, warmup):
    """Set the initial data, capture the `steps`-step graph (hw_prepare_advance, not
    timed), `warmup` untimed steps, then the timed `steps` steps."""
    spec = w.spec
    s = B.Solver(spec, precision=precision, kernel=kernel)
    s.set_state(w.u0, w.v0)
    if warmup:
        B.hw_prepare_advance(s.h, warmup)
    B.hw_advance(s.h, warmup)
    B.hw_prepare_advance(s.h, steps)
    torch.cuda.synchronize()
    elapsed, ev_ms = timed_advance(torch, B, s.h, steps, 0)
    return s, elapsed, ev_ms


def l2_errors(torch, W, w, s, t_final):
    """nodal L2 error of the value coefficient against the exact radial solution"""
    u, _ = s.get_state()
    val = u[:, 0]
    spec = w.spec
    pts = torch.as_tensor(spec.points(W.PRIMAL), device="cuda")
    ex = torch.empty_like(val)
    chunk = 1 << 21
    for a in range(0, pts.shape[0], chunk):
        ex[a:a + chunk] = w.exact(t_final, points=pts[a:a + chunk], xp=torch)
    h3 = spec.h(0) * spec.h(1) * spec.h(2)
    diff = val - ex
    err = math.sqrt(h3 * float((diff * diff).sum()))
    ref = math.sqrt(h3 * float((ex * ex).sum()))
    return err, err / ref, val


def physical_cores():
    """(physical cores, logical CPUs) of the host, from /proc/cpuinfo."""
    logical = os.cpu_count() or 1
    try:
        pairs = set()
        phys = core = None
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("physical id"):
                    phys = line.split(":")[1].strip()
                elif line.startswith("core id"):
                    core = line.split(":")[1].strip()
                elif not line.strip() and phys is not None and core is not None:
                    pairs.add((phys, core))
                    phys = core = None
        if phys is not None and core is not None:
            pairs.add((phys, core))
        return (len(pairs) or logical), logical
    except OSError:
        return logical, logical


def cpu_baseline(W, layers, n, threads=None):
    """The FP64 oracle (as it stands) on a bounded sample of the same workload: the
    first `layers` z-layers of cells of the n^3 grid, one primal -> dual half step."""
    import oracle
    w = W.c4_3d(n=4)  # for the pulse parameters only
    centres, amps, sigma = w.meta["centres"], w.meta["amps"], w.meta["sigma"]
    h = 1.0 / n
    dt = 0.9 * h
    # slab: x, y periodic; z = [0, layers*h]; its primal nodes are the real grid's
    # first layers+1 node layers, the data uses minimum images in every dimension
    box = W.make_spec(3, 3, [n, n, layers], [0.0, 0.0, 0.0], [1.0, 1.0, layers * h], 1.0,
                      dt=dt, bc=[W.PERIODIC, W.PERIODIC, W.DIRICHLET])
    terms = []
    for x0, A in zip(centres, amps):
        def term(i, x, L, hh, x0=x0, A=A):
            t = W.gaussian_derivs(x, x0[i], sigma, L, hh, period=1.0)
            return t * A if i == 0 else t
        terms.append(term)
    u = W.separable_nodal(box, W.PRIMAL, 4, terms)
    v = np.zeros((box.nodes(W.PRIMAL), 27))
    if threads is None:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    p = oracle.make_problem(3, 3, box.n, box.xl, box.xr, 1.0, dt, box.bc, W.DISS_FULL)
    t0 = time.perf_counter()
    uo, _ = oracle.diss_half(p, oracle.DUAL, u, v, nthreads=threads)
    el = time.perf_counter() - t0
    cells = uo.shape[0]
    try:
        model = subprocess.run(["sh", "-c", "grep -m1 'model name' /proc/cpuinfo | cut -d: -f2"],
                               capture_output=True, text=True).stdout.strip()
    except Exception:
        model = ""
    return {"value": cells / el, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{cells} cells ({layers} z-layers of the {n}^3 grid), one primal->dual "
                      f"half step, FP64, {el:.1f} s, CPU: {model}"}


def rel_chunked(torch, a, b):
    """relative L2 norm of a - b over every entry (chunked)"""
    num = den = 0.0
    step = 1 << 22
    for k in range(0, a.shape[0], step):
        num += float(((a[k:k + step] - b[k:k + step]) ** 2).sum())
        den += float((b[k:k + step] ** 2).sum())
    return math.sqrt(num / den)


def accuracy_leg(torch, B, W, w, steps, kernel):
    """The workload's own length, untimed: FP32 and FP64 forms advanced `steps` steps from
    the initial data; the value coefficient against the exact radial solution (nodal L2),
    and the FP32 state against the FP64 state over every coefficient, u and v apart."""
    out = {}
    states = {}
    for prec, name in ((B.HW_FP64, "fp64"), (B.HW_FP32, "fp32")):
        s = B.Solver(w.spec, precision=prec, kernel=kernel)
        s.set_state(w.u0, w.v0)
        s.advance(steps)
        err, rel, _ = l2_errors(torch, W, w, s, steps * w.spec.dt)
        out[f"{name}_value_rel"] = rel
        out[f"{name}_value_abs"] = err
        states[name] = s.get_state()
        s.close()
    (u32, v32), (u64, v64) = states["fp32"], states["fp64"]
    out["fp32_vs_fp64_value_rel"] = rel_chunked(torch, u32[:, :1], u64[:, :1])
    out["fp32_vs_fp64_all_u_coefficients_rel"] = rel_chunked(torch, u32, u64)
    out["fp32_vs_fp64_all_v_coefficients_rel"] = rel_chunked(torch, v32, v64)
    out["steps"] = steps
    out["t_final"] = steps * w.spec.dt
    del states, u32, v32, u64, v64
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the Hermite half step shards by slabs with a "
              "one-node halo exchange, which this library does not implement; use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1802_05246_amd import binding as B
    from paper_1802_05246_amd import workloads as W

    B.lib()
    if args.copy_calibration:
        log("[bench] copy calibration")
        copy_calibration(torch)
    kernel = {"auto": B.HW_KERNEL_AUTO, "composed": B.HW_KERNEL_COMPOSED, "generic": B.HW_KERNEL_GENERIC,
              "tiled": B.HW_KERNEL_TILED}[args.kernel]
    n = args.n
    log(f"[bench] building {n}^3 m=3 pulse data on the GPU")
    w = W.c4_3d(n=n, device="cuda")
    spec = w.spec
    cells_per_step = 2 * spec.nodes(W.PRIMAL)  # two half steps, periodic: n^3 nodes each
    K, Wm = args.steps, args.warmup

    # FP32 form (the metric's value)
    log(f"[bench] fp32 form: warmup {Wm}, timed {K} steps")
    s32, el32, ev32 = run_form(torch, B, W, w, B.HW_FP32, kernel, K, Wm)
    rate32 = cells_per_step * K / el32
    t_final = (K + Wm) * spec.dt
    err32 = rel32 = None
    if not args.no_error:
        err32, rel32, val32 = l2_errors(torch, W, w, s32, t_final)
    s32.close()

    # FP64 form
    K64 = args.fp64_steps or K
    log(f"[bench] fp64 form: warmup {Wm}, timed {K64} steps")
    s64, el64, ev64 = run_form(torch, B, W, w, B.HW_FP64, kernel, K64, Wm)
    rate64 = cells_per_step * K64 / el64
    err64 = rel64 = diff_32_64 = None
    if not args.no_error:
        if K64 == K:
            err64, rel64, val64 = l2_errors(torch, W, w, s64, t_final)
            diff_32_64 = float(torch.linalg.norm(val32 - val64) / torch.linalg.norm(val64))
        else:
            err64, rel64, _ = l2_errors(torch, W, w, s64, (K64 + Wm) * spec.dt)
    s64.close()

    # the LDS-tiled kernel in FP32 (the BF16 form's kernel), reported beside the default
    # composed-map kernel
    tiled32 = None
    if not args.no_tiled and args.kernel == "auto":
        log(f"[bench] tiled fp32 kernel: warmup {Wm}, timed {K} steps")
        sc, elc, evc = run_form(torch, B, W, w, B.HW_FP32, B.HW_KERNEL_TILED, K, Wm)
        tiled32 = {"value": cells_per_step * K / elc, "unit": "cell-updates/s", "steps": K,
                   "ms_per_step": elc / K * 1e3, "kernel_avg_ms": evc / (2 * K)}
        if not args.no_error:
            errc, relc, _ = l2_errors(torch, W, w, sc, t_final)
            tiled32.update({"l2_abs": errc, "l2_rel": relc})
        sc.close()

    # BF16-operand form (FP32 storage and accumulation), reported beside the others
    bf16 = None
    if not args.no_bf16:
        log(f"[bench] bf16-operand form: warmup {Wm}, timed {K} steps")
        s16, el16, ev16 = run_form(torch, B, W, w, B.HW_BF16, B.HW_KERNEL_TILED, K, Wm)
        bf16 = {"value": cells_per_step * K / el16, "unit": "cell-updates/s", "steps": K,
                "ms_per_step": el16 / K * 1e3, "kernel_avg_ms": ev16 / (2 * K)}
        if not args.no_error:
            err16, rel16, val16 = l2_errors(torch, W, w, s16, t_final)
            bf16.update({"l2_abs": err16, "l2_rel": rel16})
            if K64 == K:
                bf16["vs_fp64_rel"] = float(torch.linalg.norm(val16 - val64) / torch.linalg.norm(val64))
        s16.close()
    accuracy = None
    if not args.no_error and args.accuracy_steps > 0:
        log(f"[bench] accuracy leg: {args.accuracy_steps} steps of the FP32 and FP64 forms (untimed)")
        accuracy = accuracy_leg(torch, B, W, w, args.accuracy_steps, kernel)
    del w
    torch.cuda.empty_cache()
    probes = None
    if not args.no_probes:
        log("[bench] peak probes: STREAM triad, matrix-core FP32 / FP64, co-execution")
        co = B.hw_probe_coexec()
        probes = {"hbm_triad_gbs": B.hw_probe_stream_triad(1 << 28),
                  "mfma_fp32_tflops": B.hw_probe_mfma(B.HW_FP32),
                  "mfma_fp64_tflops": B.hw_probe_mfma(B.HW_FP64),
                  "coexec_ms": {"products": co[0], "vector_fmas": co[1], "both": co[2],
                                "overlap_frac": (co[0] + co[1] - co[2]) / min(co[0], co[1])},
                  "note": "attainable peaks measured on this GPU (triad over three 2 GiB FP64 arrays; "
                          "independent 16x16x4 matrix-core products); coexec: the same products and "
                          "independent FP32 FMAs timed alone and together in every wave "
                          "(overlap_frac 1: fully overlapped, 0: taking turns)"}

    # roofline of the dominant kernel (the half-step kernel of the FP32 form)
    launches = 2 * K
    avg_ms = ev32 / launches
    cells_per_launch = spec.nodes(W.PRIMAL)
    recorded = args.kernel in ("auto", "composed")  # the FP32 kernel the traffic record belongs to
    flops_launch = FLOPS_PER_CELL * cells_per_launch
    bytes_launch = BYTES_PER_CELL["fp32"] * cells_per_launch
    ach_tflops = flops_launch / (avg_ms * 1e-3) / 1e12
    ach_gbs = bytes_launch / (avg_ms * 1e-3) / 1e9
    exe_tflops = EXECUTED_FLOPS_PER_CELL * cells_per_launch / (avg_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": round(ach_tflops, 2),
            "peak": PEAKS_TFLOPS["fp32"], "unit": "TFLOP/s",
            "frac": round(ach_tflops / PEAKS_TFLOPS["fp32"], 4), "traffic": traffic_bytes() if (recorded and n == 256) else None,
            "achieved_counts": "algorithmic flops (48 272 per cell-update, the factored method of the "
                               "paper counted per cell): an algorithm-equivalent rate",
            "executed_tflops": round(exe_tflops, 2),
            "executed_frac": round(exe_tflops / PEAKS_TFLOPS["fp32"], 4),
            "executed_counts": f"{EXECUTED_FLOPS_PER_CELL} flops per cell-update executed by the composed-map "
                               "kernel (matrix-core multiply-adds incl. padding, butterfly additions)",
            "mfma_busy_frac": mfma_busy() if (recorded and n == 256) else None,
            "kernel_avg_ms": round(avg_ms, 4), "hbm_algorithmic_gbs": round(ach_gbs, 1),
            "hbm_frac": round(ach_gbs / HBM_PEAK_GBS, 4)}
    if probes:
        roof["measured_peaks"] = probes
        roof["frac_of_measured_fp32_mfma"] = round(ach_tflops / probes["mfma_fp32_tflops"], 4)

    cpu = None
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline: oracle on {args.cpu_layers} z-layers")
        cpu = cpu_baseline(W, args.cpu_layers, n)
        phys, logical = physical_cores()
        cpu["physical_cores"] = phys
        cpu["logical_cpus"] = logical
        cpu["omp_num_threads_env"] = os.environ.get("OMP_NUM_THREADS")
        if args.cpu_layers_1t > 0:
            log(f"[bench] cpu baseline, one thread: oracle on {args.cpu_layers_1t} z-layers")
            one = cpu_baseline(W, args.cpu_layers_1t, n, threads=1)
            cpu["value_1thread"] = one["value"]
            cpu["sample_1thread"] = one["sample"]

    out = {
        "metric": METRIC, "value": rate32, "unit": "cell-updates/s", "n_gpus": 1, "steps": K,
        "warmup": Wm, "ms_per_step": el32 / K * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"3-D dissipative Hermite (modified first step), m=3, periodic "
                               f"unit cube {n}^3, c dt/h = 0.9, 8 Gaussian pulses sigma 0.05, v0 = 0",
                   "n": n, "m": 3, "cfl": 0.9, "cells_per_step": cells_per_step,
                   "kernel": args.kernel},
        "l2_error": {"fp32_abs": err32, "fp32_rel": rel32, "fp64_abs": err64, "fp64_rel": rel64,
                     "fp32_vs_fp64_rel": diff_32_64, "t_final": t_final,
                     "against": "exact radial solution, value coefficient at the primal nodes"},
        "fp64_form": {"value": rate64, "unit": "cell-updates/s", "steps": K64,
                      "ms_per_step": el64 / K64 * 1e3, "speedup_fp32_over_fp64": rate32 / rate64,
                      "kernel_avg_ms": ev64 / (2 * K64)},
        "tiled_fp32_form": tiled32,
        "bf16_form": bf16,
        "accuracy_at_workload_length": accuracy,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
