#!/usr/bin/env python3
"""Throughput of the RKDG time step with the jump filter on one MI355X.

Workload (default): 1D Euler, Shu-Osher Mach-3 shock into a density wave,
20000 cells on [-5, 5], P^2 modal Legendre, outflow ends, SSP-RK3 at CFL
0.1, hybrid limiter with the jump filter as low-order limiter after every
stage, FP64.  A step is one full SSP-RK3 step (3 stages, each the fused
residual + RK combination + filter/hybrid kernels, plus the device-side CFL
reduction and time-step control), replayed from a HIP graph.

Metric: DOF-updates per second per RK stage = DOFs x 3 x steps / wall time,
with the inputs resident in HBM before the timed region starts.

Prints ONE JSON line.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "DOF-updates/s per RK stage and % HBM roofline, FP32 vs FP64, batched vs single"


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bytes_per_dof_update(k: int, precision: int) -> float:
    """Algorithmic HBM bytes per DOF per stage: each SSP-RK3 stage reads the
    stage input, reads u^n (stages 2 and 3) and writes the output, i.e. 8/3
    state passes per stage on average; FP64 stores 8 B per DOF, the mixed
    form 8 B for mode 0 and 4 B for every other mode."""
    per_dof = 8.0 if precision == 0 else (8.0 + 4.0 * k) / (k + 1)
    return 8.0 / 3.0 * per_dof


def run_gpu(dg, torch, w, precision: int, steps: int, warmup: int):
    mesh = dg.make_mesh(1, (w.n,), (w.lo,), (w.hi,), (dg.DG_BC_OUTFLOW, dg.DG_BC_OUTFLOW))
    opt = dg.make_options(precision=precision, filter=dg.DG_FILTER_HYBRID, cfl=w.cfl,
                          gamma=w.gamma)
    s = dg.Solver(mesh, w.k, dg.DG_EQ_EULER, opt)
    s.set_state(w.u0)
    if warmup:
        dg.dg_run(s.h, 1e30, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = dg.dg_run(s.h, 1e30, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert rep.steps == warmup + steps, (rep.steps, warmup, steps)
    return s, rep, wall


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--cells", type=int, default=20000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-variants", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the per-GPU throughput at N=1 is the figure it reports).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import dg_inputs as I
    import paper_2407_19169_amd as dg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w = I.shu_osher(args.cells, 2)
    ndof = 3 * (w.k + 1) * w.n
    log(f"workload: Shu-Osher {w.n} cells P{w.k} hybrid, {ndof} DOFs; warmup {args.warmup}, "
        f"steps {args.steps}")

    s, rep, wall = run_gpu(dg, torch, w, dg.DG_PREC_FP64, args.steps, args.warmup)
    value = ndof * 3 * args.steps / wall
    log(f"fp64: {value:.4e} DOF-updates/s, {1e3 * wall / args.steps:.4f} ms/step, "
        f"troubled cells {rep.troubled_cells}")

    # Dominant kernel: the fused stage + hybrid pass A kernel, timed with HIP
    # events on the stream it runs on.
    dt = rep.dt_max
    durs = [dg.dg_time_kernel(s.h, st, dt, 50) for st in range(3)]
    avg_us = sum(durs) / 3.0
    bytes_launch = bytes_per_dof_update(w.k, 0) * ndof
    achieved = bytes_launch / (avg_us * 1e-6) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                "kernel": "stage1d_kernel<EULER,2,double,2> (fused residual + RK + hybrid pass A)",
                "avg_launch_us": round(avg_us, 3),
                "per_stage_us": [round(d, 3) for d in durs],
                "bytes_per_launch": int(bytes_launch),
                "note": "20000-cell state (1.4 MB) is cache-resident: latency-bound, not HBM-bound"}
    s.close()

    variants = {}
    if not args.no_variants:
        sm, repm, wallm = run_gpu(dg, torch, w, dg.DG_PREC_MIXED, args.steps, args.warmup)
        vm = ndof * 3 * args.steps / wallm
        variants["mixed_fp32_bulk_fp64_mode0"] = {
            "value": vm, "ms_per_step": 1e3 * wallm / args.steps,
            "ratio_vs_fp64": vm / value}
        log(f"mixed: {vm:.4e} DOF-updates/s")
        sm.close()

    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O

        P = O.problem1d(O.EULER, w.k, w.n, w.lo, w.hi, bc=(O.OUTFLOW, O.OUTFLOW),
                        filter=O.FILTER_HYBRID, cfl=w.cfl)
        t0 = time.perf_counter()
        O.run1d(P, w.u0, 1e30, 10)
        probe = time.perf_counter() - t0
        nsteps = max(10, int(args.cpu_seconds / max(probe / 10, 1e-6)))
        t0 = time.perf_counter()
        O.run1d(P, w.u0, 1e30, nsteps)
        tc = time.perf_counter() - t0
        cpu = {"value": ndof * 3 * nsteps / tc, "unit": "DOF-updates/s",
               "cores": int(O.lib().dgref_num_threads()), "kind": "oracle",
               "sample": f"same workload, first {nsteps} steps ({tc:.1f} s)"}
        log(f"cpu oracle: {cpu['value']:.4e} DOF-updates/s on {cpu['cores']} threads")

    out = {
        "metric": METRIC, "value": value, "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "1D Euler Shu-Osher (Mach-3 shock into rho=1+0.2 sin 5x), "
                               f"{w.n} cells on [-5,5], P2, outflow, SSP-RK3 CFL 0.1, hybrid "
                               "limiter with jump filter, FP64",
                   "cells": w.n, "degree": w.k, "dofs": ndof, "precision": "fp64"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
