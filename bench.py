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
# HBM bytes per launch of the headline stage kernel (20000 cells, P2, FP64,
# hybrid pass A), from rocprofv3 FETCH_SIZE and WRITE_SIZE over the
# back-to-back timing launches, each scaled by what the counter reads for a
# plain 1 GiB device copy (FETCH x2.0, WRITE x1.0); the summary with the
# commands is profiles/stage1d_headline_traffic.md.  Set to None when that
# kernel changes until the counters are taken again.
HEADLINE_TRAFFIC_BYTES = (1700.9 * 2.0 + 1565.4 * 1.0) * 1024
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


def _timed_run(dg, torch, s, steps: int, warmup: int):
    if warmup:
        dg.dg_run(s.h, 1e30, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = dg.dg_run(s.h, 1e30, steps)
    torch.cuda.synchronize()
    return rep, time.perf_counter() - t0


def sweep_1d(dg, torch, I, sizes, steps: int):
    """Jump filter on HBM-sized 1D states (Shu-Osher profile on n cells, P2):
    step throughput of dg_run, whose kernel runs all three stages of a step
    in one pass, that kernel's bandwidth (2 state passes per step), the same
    time against the stage-wise denominator of 8/3 passes per stage (labelled
    as such), and the single-stage kernel (stage + filter) per launch."""
    out = []
    for n in sizes:
        w = I.shu_osher(n, 2)
        ndof = 3 * (w.k + 1) * n
        for prec in (dg.DG_PREC_FP64, dg.DG_PREC_MIXED):
            mesh = dg.make_mesh(1, (n,), (w.lo,), (w.hi,), (dg.DG_BC_OUTFLOW, dg.DG_BC_OUTFLOW))
            opt = dg.make_options(precision=prec, filter=dg.DG_FILTER_JUMP, cfl=w.cfl)
            s = dg.Solver(mesh, w.k, dg.DG_EQ_EULER, opt)
            s.set_state(w.u0)
            rep, wall = _timed_run(dg, torch, s, steps, 2)
            durs = [dg.dg_time_kernel(s.h, st, rep.dt_max, 20) for st in range(3)]
            avg = sum(durs) / 3.0
            b = bytes_per_dof_update(w.k, prec) * ndof
            gbs = b / (avg * 1e-6) / 1e9
            # the kernel dg_run uses: all three stages of a step in one pass
            # (reads u^n, writes u^{n+1}: 2 state passes per step)
            step_us = dg.dg_time_kernel(s.h, 6, rep.dt_max, 20)
            state_bytes = b * 3.0 / 8.0   # one pass over the state
            step_gbs = 2.0 * state_bytes / (step_us * 1e-6) / 1e9
            equiv_gbs = 3.0 * b / (step_us * 1e-6) / 1e9
            out.append({"cells": n, "precision": "fp64" if prec == 0 else "mixed",
                        "dof_updates_per_s": ndof * 3 * steps / wall,
                        "ms_per_step": 1e3 * wall / steps,
                        "stage_kernel_us": round(avg, 2), "stage_kernel_GBps": round(gbs, 1),
                        "stage_kernel_hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                        "step_kernel_us": round(step_us, 2), "step_kernel_GBps": round(step_gbs, 1),
                        "step_kernel_hbm_frac": round(step_gbs / HBM_PEAK_GBS, 4),
                        "step_kernel_stagewise_equiv_GBps": round(equiv_gbs, 1)})
            log(f"1D sweep n={n} {out[-1]['precision']}: {out[-1]['dof_updates_per_s']:.3e} "
                f"DOF-updates/s; stage kernel {avg:.1f} us = {gbs:.0f} GB/s; fused step "
                f"{step_us:.1f} us = {step_gbs:.0f} GB/s ({equiv_gbs:.0f} GB/s stage-wise)")
            s.close()
        del w
    return out


def bench_2d(dg, torch, I, w, mesh, prec: int, filt: int, steps: int, basis: int = 0):
    """A 2D workload: step throughput and, per stage, the residual and filter
    kernel times against the stage's algorithmic bytes.  basis 1: the P^k
    space (the modes p + q <= k are the DOFs)."""
    nm = (w.k + 1) ** 2 if basis == 0 else (w.k + 1) * (w.k + 2) // 2
    ndof = 4 * nm * w.nx * w.ny
    opt = dg.make_options(precision=prec, filter=filt, cfl=w.cfl, basis=basis)
    s = dg.Solver(mesh, w.k, dg.DG_EQ_EULER, opt)
    s.set_state(w.u0)
    rep, wall = _timed_run(dg, torch, s, steps, 2)
    res = [dg.dg_time_kernel(s.h, st, rep.dt_max, 10) for st in range(3)]
    fil = [dg.dg_time_kernel(s.h, 3 + st, rep.dt_max, 10) for st in range(3)]
    s.close()
    per_dof = 8.0 if prec == 0 else (8.0 + 4.0 * (nm - 1)) / nm
    b = 8.0 / 3.0 * per_dof * ndof
    stage_us = (sum(res) + sum(fil)) / 3.0
    gbs = b / (stage_us * 1e-6) / 1e9
    return {"dofs": ndof, "space": "Q^k" if basis == 0 else "P^k",
            "precision": "fp64" if prec == 0 else "mixed", "status": rep.status,
            "dof_updates_per_s": ndof * 3 * steps / wall, "ms_per_step": 1e3 * wall / steps,
            "residual_kernel_us": round(sum(res) / 3, 2), "filter_kernel_us": round(sum(fil) / 3, 2),
            "stage_GBps": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}


def bench_batch(dg, torch, I, steps: int):
    """4096 seeded Riemann problems (256..8192 cells, P1-P3), mixed
    precision, jump filter + positivity limiter, one persistent launch."""
    spec = I.batched_riemann_spec(4096, 4001)
    states = I.batched_riemann_states(spec)
    probs = [(int(spec.n[i]), int(spec.k[i]), -1.0, 1.0, dg.DG_BC_OUTFLOW, dg.DG_BC_OUTFLOW)
             for i in range(len(spec.n))]
    ndof = int(sum(3 * (k + 1) * n for n, k, *_ in probs))
    b = dg.Batch(probs, dg.make_options(precision=dg.DG_PREC_MIXED, filter=dg.DG_FILTER_JUMP,
                                         cfl=0.1, positivity=1))
    b.set_state(states)
    tune = json.loads(b.tune(3))
    b.set_state(states)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = b.run(steps, check=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    done = sum(int(r.steps) for r in reps)
    upd = sum(3 * (k + 1) * n * int(r.steps) * 3 for (n, k, *_), r in zip(probs, reps))
    # stage-wise algorithmic bytes: 8/3 state passes per stage at each
    # problem's own mixed-precision bytes per DOF (retried steps not
    # counted).  The kernel runs the three stages of a step in one pass, so
    # it moves 2 passes per step: the step-wise figure is 1/4 of this.
    nbytes = sum(3 * (k + 1) * n * int(r.steps) * 3 * bytes_per_dof_update(k, 1)
                 for (n, k, *_), r in zip(probs, reps))
    b.close()
    gbs = nbytes / wall / 1e9
    return {"problems": len(probs), "dofs": ndof, "steps_requested": steps,
            "steps_done": done, "failed": sum(1 for r in reps if r.status == -4),
            "retries": sum(int(r.restarts) for r in reps),
            "dof_updates_per_s": upd / wall, "wall_s": wall,
            "stagewise_equiv_GBps": round(gbs, 1), "step_traffic_GBps": round(gbs / 4.0, 1),
            "step_traffic_hbm_frac": round(gbs / 4.0 / HBM_PEAK_GBS, 4),
            "schedule": tune.get("best")}


def _dmr_mesh(dg, I, np, nx, ny, k):
    wd = I.double_mach(nx, ny, k)
    post, pre = I.conserved2d(*wd.extra["post"]), I.conserved2d(1.4, 0.0, 0.0, 1.0)
    speed = wd.extra["shock_speed"] / np.sin(np.pi / 3)
    mesh = dg.make_mesh(2, (nx, ny), (0.0, 0.0), (4.0, 1.0),
                        (dg.DG_BC_DIRICHLET, dg.DG_BC_OUTFLOW, 4, 5),
                        dirichlet=[list(post)] * 4, shock_x0=1 / 6, shock_speed=speed,
                        post=list(post), pre=list(pre))
    return wd, mesh


def run_only(args, dg, torch, I, np) -> int:
    if args.only == "sweep":
        r = sweep_1d(dg, torch, I, [int(x) for x in args.sweep.split(",") if x], args.steps)
    elif args.only == "vortex":
        wv = I.vortex2d(1024, 2, seed=3001)
        mesh = dg.make_mesh(2, (1024, 1024), (0.0, -5.0), (10.0, 5.0), (0, 0, 0, 0))
        r = [bench_2d(dg, torch, I, wv, mesh, p, dg.DG_FILTER_JUMP, args.steps, basis=b)
             for p in (0, 1) for b in (0, 1)]
    elif args.only == "dmr":
        wd, mesh = _dmr_mesh(dg, I, np, 4096, 1024, 3)
        r = [bench_2d(dg, torch, I, wd, mesh, dg.DG_PREC_MIXED, dg.DG_FILTER_JUMP, args.steps, basis=b)
             for b in (0, 1)]
    elif args.only == "copy":
        # reference for hardware traffic counters: a plain 1 GiB device copy
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        r = {"bytes_read_per_copy": x.numel() * 8, "bytes_written_per_copy": y.numel() * 8}
    else:
        r = bench_batch(dg, torch, I, args.steps)
    print(json.dumps({"only": args.only, "result": r}), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--cells", type=int, default=20000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--only", choices=["sweep", "vortex", "dmr", "batch", "copy"], default=None,
                    help="run one supplementary workload alone and print its figures "
                         "(for profiler runs); no headline line")
    ap.add_argument("--sweep", default="1000000,4000000,16000000",
                    help="1D cell counts of the HBM sweep (comma separated, empty: skip; "
                         "multiples of 10 keep the initial shock on a cell interface)")
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
    if args.only:
        return run_only(args, dg, torch, I, np)
    w = I.shu_osher(args.cells, 2)
    ndof = 3 * (w.k + 1) * w.n
    log(f"workload: Shu-Osher {w.n} cells P{w.k} hybrid, {ndof} DOFs; warmup {args.warmup}, "
        f"steps {args.steps}")

    s, rep, wall = run_gpu(dg, torch, w, dg.DG_PREC_FP64, args.steps, args.warmup)
    value = ndof * 3 * args.steps / wall
    log(f"fp64: {value:.4e} DOF-updates/s, {1e3 * wall / args.steps:.4f} ms/step, "
        f"troubled cells {rep.troubled_cells}")

    # Dominant kernel: the fused stage + hybrid pass A kernel, timed with HIP
    # events on the stream it runs on (stage 2 in its variant that also runs
    # the next step's control in its last workgroup, as dg_run launches it).
    dt = rep.dt_max
    durs = [dg.dg_time_kernel(s.h, st, dt, 50) for st in range(3)]
    avg_us = sum(durs) / 3.0
    bytes_launch = bytes_per_dof_update(w.k, 0) * ndof
    achieved = bytes_launch / (avg_us * 1e-6) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                "traffic": None if HEADLINE_TRAFFIC_BYTES is None else int(HEADLINE_TRAFFIC_BYTES),
                "kernel": "stage1d_kernel<EULER,2,double,2> (fused residual + RK + hybrid pass A; "
                          "stage 2 also runs the step control)",
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
        sizes = [int(x) for x in args.sweep.split(",") if x]
        if sizes:
            variants["sweep_1d_fused_jump_filter"] = sweep_1d(dg, torch, I, sizes, 20)
        wv = I.vortex2d(1024, 2, seed=3001)
        mesh = dg.make_mesh(2, (1024, 1024), (0.0, -5.0), (10.0, 5.0), (0, 0, 0, 0))
        for prec in (dg.DG_PREC_FP64, dg.DG_PREC_MIXED):
            r = bench_2d(dg, torch, I, wv, mesh, prec, dg.DG_FILTER_JUMP, 20)
            variants[f"vortex2d_1024_q2_{r['precision']}"] = r
            log(f"vortex 1024^2 Q2 {r['precision']}: {r['dof_updates_per_s']:.3e} DOF-updates/s, "
                f"stage {r['stage_GBps']} GB/s")
        r = bench_2d(dg, torch, I, wv, mesh, dg.DG_PREC_MIXED, dg.DG_FILTER_JUMP, 20, basis=1)
        variants["vortex2d_1024_p2_mixed"] = r
        log(f"vortex 1024^2 P2 mixed: {r['dof_updates_per_s']:.3e} DOF-updates/s, "
            f"stage {r['stage_GBps']} GB/s")
        del wv
        wd, meshd = _dmr_mesh(dg, I, np, 4096, 1024, 3)
        for basis, name in ((0, "q3"), (1, "p3")):
            r = bench_2d(dg, torch, I, wd, meshd, dg.DG_PREC_MIXED, dg.DG_FILTER_JUMP, 10, basis=basis)
            variants[f"double_mach_4096x1024_{name}_mixed"] = r
            log(f"double Mach 4096x1024 {name.upper()} mixed: {r['dof_updates_per_s']:.3e} "
                f"DOF-updates/s, stage {r['stage_GBps']} GB/s")
        del wd
        rb = bench_batch(dg, torch, I, 200)
        variants["batched_riemann_4096_mixed_pp"] = rb
        log(f"batched 4096 problems: {rb['dof_updates_per_s']:.3e} DOF-updates/s "
            f"({rb['stagewise_equiv_GBps']} GB/s stage-wise, {rb['step_traffic_GBps']} GB/s "
            f"moved), {rb['failed']} failed, {rb['retries']} retries")

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
