#!/usr/bin/env python3
"""Throughput of the RKDG time step with the jump filter on one MI355X.

Headline workload: 2D Euler double Mach reflection (Mach-10 shock inclined
60 degrees into (rho, p) = (1.4, 1), reflecting wall, exact moving shock on
the top boundary), 4096 x 1024 cells on [0,4] x [0,1], Q^3 tensor Legendre
(16 modes x 4 variables = 268M DOFs), SSP-RK3 at CFL 0.1, hybrid limiter
(Algorithm 1: troubled-cell indicator + jump filter with the printed
coefficient) and the positivity limiter after every stage, FP64.  A step is
one SSP-RK3 step (3 stages, each: residual + RK combination, hybrid pass A,
blend of the troubled cells, positivity limiter on the listed cells; plus the
device-side CFL reduction and time-step control), replayed from a HIP graph.

Metric: DOF-updates per second per RK stage = DOFs x 3 x steps / wall time,
with the inputs resident in HBM before the timed region starts.

Variants (each its own workload, same metric): the mixed form of the
headline (FP32 bulk, FP64 mode 0 and checks); the 1D Burgers (200 cells),
Shu-Osher (20000 cells), 2D vortex and four-quadrant (1024^2, Q^2) and
4096-problem batched Riemann workloads; a 1D HBM-size sweep.  Each gives the
mixed form's relative L1 of the cell averages against the FP64 form.

Prints ONE JSON line.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "DOF-updates/s per RK stage and % HBM roofline, FP32 vs FP64, batched vs single"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bytes_per_dof_update(nmodes: int, precision: int) -> float:
    """Algorithmic HBM bytes per DOF per stage: each SSP-RK3 stage reads the
    stage input, reads u^n (stages 2 and 3) and writes the output, i.e. 8/3
    state passes per stage on average; FP64 stores 8 B per DOF, the mixed
    form 8 B for mode 0 and 4 B for every other mode."""
    per_dof = 8.0 if precision == 0 else (8.0 + 4.0 * (nmodes - 1)) / nmodes
    return 8.0 / 3.0 * per_dof


def rel_l1(a, b):
    """Relative L1 of the cell averages, per variable (mode axis 1)."""
    import numpy as np

    return [float(np.sum(np.abs(a[v, 0] - b[v, 0])) / max(np.sum(np.abs(b[v, 0])), 1e-300))
            for v in range(a.shape[0])]


def timed_run(dg, torch, s, steps: int, warmup: int, t_end: float = 1e30):
    """Warm-up steps, then the timed dg_run; returns its report, its wall
    time and the steps it took (the report counts the handle's steps)."""
    steps0 = 0
    if warmup:
        steps0 = int(dg.dg_run(s.h, t_end, warmup).steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = dg.dg_run(s.h, t_end, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rep.timed_steps = int(rep.steps) - steps0
    return rep, wall


def src_digest() -> str:
    """Digest of the 2D kernel source the traffic counters were taken on."""
    h = hashlib.sha256()
    for f in ("dg2d.hip", "dg_kernels.h", "dg_common.h"):
        with open(os.path.join(ROOT, "paper_2407_19169_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(key: str):
    """HBM bytes per stage of the headline's kernels from the rocprofv3
    counter summary (FETCH_SIZE, WRITE_SIZE per dispatch, scaled by a plain
    copy's counts), or None when none was taken on the current source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh).get(key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("src_digest") != src_digest():
        return None
    return rec.get("bytes_per_stage")


# ---------------------------------------------------------------- 2D ----
def dmr_setup(dg, I, np, nx, ny, k):
    wd = I.double_mach(nx, ny, k)
    post, pre = I.conserved2d(*wd.extra["post"]), I.conserved2d(1.4, 0.0, 0.0, 1.0)
    speed = wd.extra["shock_speed"] / math.sin(math.pi / 3)
    mesh = dg.make_mesh(2, (nx, ny), (0.0, 0.0), (4.0, 1.0),
                        (dg.DG_BC_DIRICHLET, dg.DG_BC_OUTFLOW, dg.DG_BC_DMR_WALL, dg.DG_BC_DMR_TOP),
                        dirichlet=[list(post)] * 4, shock_x0=1 / 6, shock_speed=speed,
                        post=list(post), pre=list(pre))
    return wd, mesh, post, pre, speed


def run_2d(dg, torch, w, mesh, prec: int, filt: int, steps: int, warmup: int, pp: int = 0,
           basis: int = 0, kernels: bool = True):
    """One 2D workload: step throughput of dg_run and, per stage, the
    residual and post-stage (filter / hybrid pass A) kernel times."""
    nm = (w.k + 1) ** 2 if basis == 0 else (w.k + 1) * (w.k + 2) // 2
    ndof = 4 * nm * w.nx * w.ny
    opt = dg.make_options(precision=prec, filter=filt, cfl=w.cfl, basis=basis, positivity=pp)
    s = dg.Solver(mesh, w.k, dg.DG_EQ_EULER, opt)
    s.set_state(w.u0)
    rep, wall = timed_run(dg, torch, s, steps, warmup)
    assert rep.timed_steps == steps, (rep.timed_steps, steps, rep.status)
    out = {"dofs": ndof, "space": "Q^k" if basis == 0 else "P^k",
           "precision": "fp64" if prec == 0 else "mixed", "status": rep.status,
           "restarts": int(rep.restarts), "troubled_cells_per_stage":
               round(rep.troubled_cells / max(3 * (steps + warmup), 1), 1),
           "dof_updates_per_s": ndof * 3 * steps / wall, "ms_per_step": 1e3 * wall / steps}
    if kernels:
        res = [dg.dg_time_kernel(s.h, st, rep.dt_max, 10) for st in range(3)]
        fil = [dg.dg_time_kernel(s.h, 3 + st, rep.dt_max, 10) for st in range(3)]
        b = bytes_per_dof_update(nm, prec) * ndof
        res_us = sum(res) / 3.0
        run_stage_us = 1e3 * wall / steps / 3.0 * 1e3
        out.update({"residual_kernel_us": round(res_us, 2),
                    "post_kernel_us": round(sum(fil) / 3, 2),
                    "per_stage_residual_us": [round(x, 2) for x in res],
                    "per_stage_post_us": [round(x, 2) for x in fil],
                    "stage_us_in_run": round(run_stage_us, 2),
                    "bytes_per_stage": int(b),
                    # the stage's compulsory traffic over the residual kernel
                    # alone, and over the whole stage as the run takes it
                    "residual_GBps": round(b / (res_us * 1e-6) / 1e9, 1),
                    "residual_hbm_frac": round(b / (res_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                    "stage_GBps": round(b / (run_stage_us * 1e-6) / 1e9, 1),
                    "hbm_frac": round(b / (run_stage_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)})
    state = s.get_state().cpu().numpy()
    s.close()
    return out, state


def variant_pair(dg, torch, w, mesh, filt, steps, warmup, pp=0, basis=0, kernels=True):
    """FP64 and mixed forms of one 2D workload, with the mixed form's L1."""
    r64, u64 = run_2d(dg, torch, w, mesh, 0, filt, steps, warmup, pp, basis, kernels)
    r32, u32 = run_2d(dg, torch, w, mesh, 1, filt, steps, warmup, pp, basis, kernels)
    r32["rel_l1_vs_fp64"] = rel_l1(u32, u64)
    return {"fp64": r64, "mixed": r32}


# ---------------------------------------------------------------- 1D ----
def run_1d(dg, torch, w, prec, filt, steps, warmup, t_end=1e30, bc=None):
    bc = bc or (dg.DG_BC_OUTFLOW, dg.DG_BC_OUTFLOW)
    mesh = dg.make_mesh(1, (w.n,), (w.lo,), (w.hi,), bc)
    s = dg.Solver(mesh, w.k, w.eq, dg.make_options(precision=prec, filter=filt, cfl=w.cfl,
                                                   gamma=w.gamma))
    s.set_state(w.u0)
    rep, wall = timed_run(dg, torch, s, steps, warmup, t_end)
    ndof = (3 if w.eq == 2 else 1) * (w.k + 1) * w.n
    done = rep.timed_steps
    r = {"dofs": ndof, "precision": "fp64" if prec == 0 else "mixed", "status": rep.status,
         "steps": done, "dof_updates_per_s": ndof * 3 * done / wall,
         "ms_per_step": 1e3 * wall / max(done, 1)}
    state = s.get_state().cpu().numpy()
    s.close()
    return r, state


def shu_osher_only(dg, torch, I, prec: int, steps: int, warmup: int):
    """The Shu-Osher problem alone (20000 cells, P2, hybrid limiter), for its
    profiles: the timed dg_run, then each stage kernel's launch time
    (dg_time_kernel: one warm-up and 50 back-to-back launches per stage)."""
    w = I.shu_osher(20000, 2)
    mesh = dg.make_mesh(1, (w.n,), (w.lo,), (w.hi,), (dg.DG_BC_OUTFLOW, dg.DG_BC_OUTFLOW))
    s = dg.Solver(mesh, w.k, w.eq, dg.make_options(precision=prec, filter=dg.DG_FILTER_HYBRID,
                                                   cfl=w.cfl, gamma=w.gamma))
    s.set_state(w.u0)
    rep, wall = timed_run(dg, torch, s, steps, warmup)
    ndof = 3 * (w.k + 1) * w.n
    done = rep.timed_steps
    per_stage = [dg.dg_time_kernel(s.h, st, rep.dt_max, 50) for st in range(3)]
    s.close()
    return {"dofs": ndof, "precision": "fp64" if prec == 0 else "mixed", "status": rep.status,
            "steps": done, "dof_updates_per_s": ndof * 3 * done / wall,
            "ms_per_step": 1e3 * wall / max(done, 1),
            "stage_kernel_us": [round(x, 2) for x in per_stage]}


def sweep_1d(dg, torch, I, sizes, steps: int):
    """Jump filter on HBM-sized 1D states (Shu-Osher profile on n cells, P2):
    dg_run runs all three stages of a step in one pass (2 state passes per
    step); also the single-stage kernel per launch."""
    out = []
    for n in sizes:
        w = I.shu_osher(n, 2)
        ndof = 3 * (w.k + 1) * n
        for prec in (0, 1):
            mesh = dg.make_mesh(1, (n,), (w.lo,), (w.hi,), (dg.DG_BC_OUTFLOW, dg.DG_BC_OUTFLOW))
            s = dg.Solver(mesh, w.k, dg.DG_EQ_EULER,
                          dg.make_options(precision=prec, filter=dg.DG_FILTER_JUMP, cfl=w.cfl))
            s.set_state(w.u0)
            rep, wall = timed_run(dg, torch, s, steps, 2)
            avg = sum(dg.dg_time_kernel(s.h, st, rep.dt_max, 20) for st in range(3)) / 3.0
            b = bytes_per_dof_update(w.k + 1, prec) * ndof
            step_us = dg.dg_time_kernel(s.h, 6, rep.dt_max, 20)
            step_gbs = 2.0 * (b * 3.0 / 8.0) / (step_us * 1e-6) / 1e9
            out.append({"cells": n, "precision": "fp64" if prec == 0 else "mixed",
                        "dof_updates_per_s": ndof * 3 * steps / wall,
                        "stage_kernel_us": round(avg, 2),
                        "stage_kernel_hbm_frac": round(b / (avg * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                        "step_kernel_us": round(step_us, 2),
                        "step_kernel_hbm_frac_moved": round(step_gbs / HBM_PEAK_GBS, 4)})
            log(f"1D sweep n={n} {out[-1]['precision']}: {out[-1]['dof_updates_per_s']:.3e}")
            s.close()
    return out


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
    upd = sum(3 * (k + 1) * n * int(r.steps) * 3 for (n, k, *_), r in zip(probs, reps))
    nbytes = sum(3 * (k + 1) * n * int(r.steps) * 3 * bytes_per_dof_update(k + 1, 1)
                 for (n, k, *_), r in zip(probs, reps))
    b.close()
    gbs = nbytes / wall / 1e9
    return {"problems": len(probs), "dofs": ndof, "steps_requested": steps,
            "failed": sum(1 for r in reps if r.status == -4),
            "retries": sum(int(r.restarts) for r in reps),
            "dof_updates_per_s": upd / wall, "wall_s": wall,
            "stagewise_equiv_GBps": round(gbs, 1),
            "step_traffic_hbm_frac": round(gbs / 4.0 / HBM_PEAK_GBS, 4),
            "schedule": tune.get("best")}


# ------------------------------------------------------------ CPU leg ----
def cpu_model() -> str:
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def cpu_baseline(I, np, seconds: float):
    """The FP64 oracle (plain C, OpenMP over cells), built here with -O3
    -march=native, on the headline's workload definition at a smaller mesh
    (the same problem and scheme; the work per DOF-update does not depend on
    the mesh size): all host threads, then one thread."""
    import ctypes as C

    import oracle as O

    tmp = tempfile.mkdtemp(prefix="dgref_o3_")
    path = O.build(out=os.path.join(tmp, "libdgref_o3.so"), opt=("-O3", "-march=native"))
    L = O.load_copy(path)
    res = {}
    for label, threads, (nx, ny), budget in (("all", 0, (512, 128), 0.7 * seconds),
                                             ("1", 1, (128, 32), 0.3 * seconds)):
        host = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
        L.dgref_set_threads(threads or host)
        nthreads = L.dgref_num_threads()
        wd = I.double_mach(nx, ny, 3)
        post, pre = I.conserved2d(*wd.extra["post"]), I.conserved2d(1.4, 0.0, 0.0, 1.0)
        speed = wd.extra["shock_speed"] / math.sin(math.pi / 3)
        P = O.problem2d(O.EULER, 3, nx, ny, 0.0, 4.0, 0.0, 1.0, bc=(3, 1, 4, 5),
                        filter=O.FILTER_HYBRID, cfl=0.1, dirichlet=[list(post)] * 4,
                        shock_x0=1 / 6, shock_speed=speed, post=post, pre=pre, pp=1)
        u = np.array(wd.u0, dtype=np.float64, order="C", copy=True)
        rep = O.Report()
        steps, t_used = 0, 0.0
        while t_used < budget or steps == 0:
            t0 = time.perf_counter()
            rc = L.dgref_run2d(C.byref(P), C.c_double(1e30), C.c_int64(1),
                               u.ctypes.data_as(C.POINTER(C.c_double)), C.byref(rep))
            t_used += time.perf_counter() - t0
            steps += 1
            if rc != 0:
                break
        ndof = 4 * 16 * nx * ny
        res[label] = {"value": ndof * 3 * steps / t_used, "threads": nthreads,
                      "sample": f"{nx}x{ny} cells, {steps} steps, {t_used:.1f} s"}
        log(f"cpu oracle ({nthreads} threads): {res[label]['value']:.4e} DOF-updates/s")
    return res


# ------------------------------------------------------------------ main ----
def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=24.0)
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--only", choices=["dmr", "sweep", "batch", "copy", "shu"], default=None,
                    help="run one workload alone and print its figures (for profiler runs)")
    ap.add_argument("--prec", type=int, default=0, help="--only dmr / shu: 0 FP64, 1 mixed")
    ap.add_argument("--sweep", default="1000000,4000000,16000000",
                    help="1D cell counts of the HBM sweep (comma separated, empty: skip)")
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

    if args.only == "copy":
        # reference for the hardware traffic counters: a plain 1 GiB device copy
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"only": "copy", "bytes_per_copy": x.numel() * 8}), flush=True)
        return 0
    if args.only == "sweep":
        r = sweep_1d(dg, torch, I, [int(x) for x in args.sweep.split(",") if x], args.steps)
        print(json.dumps({"only": "sweep", "result": r}), flush=True)
        return 0
    if args.only == "shu":
        r = shu_osher_only(dg, torch, I, args.prec, args.steps, args.warmup)
        print(json.dumps({"only": "shu", "result": r}), flush=True)
        return 0
    if args.only == "batch":
        print(json.dumps({"only": "batch", "result": bench_batch(dg, torch, I, args.steps)}),
              flush=True)
        return 0

    # ---- headline: double Mach reflection, 4096 x 1024, Q3, hybrid + PP ----
    nx, ny, k = 4096, 1024, 3
    wd, mesh, post, pre, speed = dmr_setup(dg, I, np, nx, ny, k)
    ndof = 4 * (k + 1) ** 2 * nx * ny
    log(f"workload: double Mach {nx}x{ny} Q{k} hybrid + positivity limiter, {ndof} DOFs; "
        f"warmup {args.warmup}, steps {args.steps}")
    head, u64 = run_2d(dg, torch, wd, mesh, args.prec if args.only else 0,
                       dg.DG_FILTER_HYBRID, args.steps, args.warmup, pp=1)
    log(f"headline: {head['dof_updates_per_s']:.4e} DOF-updates/s, {head['ms_per_step']:.3f} "
        f"ms/step, stage kernels {head['residual_kernel_us']} + {head['post_kernel_us']} us")
    if args.only == "dmr":
        print(json.dumps({"only": "dmr", "result": head}), flush=True)
        return 0
    value = head["dof_updates_per_s"]
    traffic = measured_traffic("double_mach_q3_fp64_hybrid_pp")
    roofline = {"bound": "hbm", "achieved": head["residual_GBps"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": head["residual_hbm_frac"],
                "traffic": traffic,
                "kernel": "stage2d_kernel<EULER,3,double> (residual, SSP-RK3 combination, and "
                          "the output's corner values for the hybrid indicator): the dominant "
                          "kernel, about 80 % of a step",
                "avg_launch_us": head["residual_kernel_us"],
                "per_stage_launch_us": head["per_stage_residual_us"],
                "bytes_per_launch": head["bytes_per_stage"],
                "unit_of_work": "one RK stage over 268,435,456 DOFs at 21.33 B/DOF (8/3 FP64 state "
                                "passes: read u^(s), read u^n in stages 2 and 3, write u^(s+1))",
                "whole_stage": {"us_in_run": head["stage_us_in_run"],
                                "GBps": head["stage_GBps"], "frac": head["hbm_frac"],
                                "note": "the same bytes over the stage as dg_run takes it: "
                                        "residual, indicator, exponents and blend of the "
                                        "troubled cells, positivity limiter, step control"},
                "indicator_kernel_us": head["post_kernel_us"]}

    variants, precision = {}, {}
    if not args.no_variants:
        r32, u32 = run_2d(dg, torch, wd, mesh, 1, dg.DG_FILTER_HYBRID, args.steps,
                          args.warmup, pp=1)
        r32["rel_l1_vs_fp64"] = rel_l1(u32, u64)
        variants["double_mach_4096x1024_q3_hybrid_pp_mixed"] = r32
        precision["double_mach_q3"] = r32["rel_l1_vs_fp64"]
        log(f"double Mach mixed: {r32['dof_updates_per_s']:.4e} DOF-updates/s, L1 "
            f"{max(r32['rel_l1_vs_fp64']):.2e}")
        del u32
        pr = variant_pair(dg, torch, wd, mesh, dg.DG_FILTER_JUMP, 10, 2, pp=1, kernels=True)
        variants["double_mach_4096x1024_q3_jump_pp"] = pr
        log(f"double Mach jump filter: fp64 {pr['fp64']['dof_updates_per_s']:.3e}, mixed "
            f"{pr['mixed']['dof_updates_per_s']:.3e}")
        del wd, u64
        wv = I.vortex2d(1024, 2, seed=3001)
        meshv = dg.make_mesh(2, (1024, 1024), (0.0, -5.0), (10.0, 5.0), (0, 0, 0, 0))
        pr = variant_pair(dg, torch, wv, meshv, dg.DG_FILTER_JUMP, 20, 2)
        variants["vortex_1024_q2_jump"] = pr
        precision["vortex_q2"] = pr["mixed"]["rel_l1_vs_fp64"]
        log(f"vortex: fp64 {pr['fp64']['dof_updates_per_s']:.3e}, mixed "
            f"{pr['mixed']['dof_updates_per_s']:.3e}")
        del wv
        wq = I.quadrant2d(1024, 2, seed=3002)
        pr = variant_pair(dg, torch, wq, meshv, dg.DG_FILTER_JUMP, 20, 2)
        variants["quadrant_1024_q2_jump"] = pr
        precision["quadrant_q2"] = pr["mixed"]["rel_l1_vs_fp64"]
        log(f"quadrant: fp64 {pr['fp64']['dof_updates_per_s']:.3e}, mixed "
            f"{pr['mixed']['dof_updates_per_s']:.3e}")
        del wq
        wb = I.burgers_sine(200, 2)
        rb64, ub64 = run_1d(dg, torch, wb, 0, 1, 100000, 0, t_end=1.5,
                            bc=(dg.DG_BC_PERIODIC, dg.DG_BC_PERIODIC))
        rb32, ub32 = run_1d(dg, torch, wb, 1, 1, 100000, 0, t_end=1.5,
                            bc=(dg.DG_BC_PERIODIC, dg.DG_BC_PERIODIC))
        rb32["rel_l1_vs_fp64"] = rel_l1(ub32, ub64)
        variants["burgers_200_p2_to_t1.5"] = {"fp64": rb64, "mixed": rb32}
        precision["burgers_p2"] = rb32["rel_l1_vs_fp64"]
        ws = I.shu_osher(20000, 2)
        rs64, us64 = run_1d(dg, torch, ws, 0, 2, 1000, 50)
        rs32, us32 = run_1d(dg, torch, ws, 1, 2, 1000, 50)
        rs32["rel_l1_vs_fp64"] = rel_l1(us32, us64)
        variants["shu_osher_20000_p2_hybrid"] = {"fp64": rs64, "mixed": rs32}
        precision["shu_osher_p2"] = rs32["rel_l1_vs_fp64"]
        log(f"Shu-Osher: fp64 {rs64['dof_updates_per_s']:.3e}, mixed "
            f"{rs32['dof_updates_per_s']:.3e}")
        sizes = [int(x) for x in args.sweep.split(",") if x]
        if sizes:
            variants["sweep_1d_fused_jump_filter"] = sweep_1d(dg, torch, I, sizes, 20)
        rb = bench_batch(dg, torch, I, 200)
        variants["batched_riemann_4096_mixed_pp"] = rb
        log(f"batched: {rb['dof_updates_per_s']:.3e} DOF-updates/s")

    cpu = None
    if not args.no_cpu_baseline:
        res = cpu_baseline(I, np, args.cpu_seconds)
        cpu = {"value": res["all"]["value"], "unit": "DOF-updates/s",
               "cores": res["all"]["threads"], "kind": "oracle",
               "sample": "FP64 oracle (C, OpenMP, gcc -O3 -march=native) on the headline "
                         f"workload at a smaller mesh: {res['all']['sample']}",
               "one_thread": res["1"]["value"], "one_thread_sample": res["1"]["sample"],
               "cpu_model": cpu_model()}

    out = {
        "metric": METRIC, "value": value, "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D Euler double Mach reflection (Mach 10, 60 degrees), "
                               f"{nx}x{ny} cells on [0,4]x[0,1], Q3 (16 modes x 4 vars), "
                               "SSP-RK3 CFL 0.1, hybrid limiter with the jump filter + "
                               "positivity limiter after every stage, FP64",
                   "cells": nx * ny, "degree": k, "dofs": ndof, "precision": "fp64",
                   "restarts": head["restarts"],
                   "troubled_cells_per_stage": head["troubled_cells_per_stage"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "precision_rel_l1_mixed_vs_fp64": precision,
        "variants": variants,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
