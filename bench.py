#!/usr/bin/env python3
"""Benchmark of the gfx950 linearized-BGK DVM solver (one JSON line).

Workload: the rough-surface channel -- a periodic cell 2H x H at 256 x 128
cells with rectangular blocks 0.2H high over half the period on both walls,
64 x 64 velocities of Eq. (nonuniform_v), delta in {0.1, 1, 10}.  One step is
the whole hot path on that input: the source iteration of Eq. (iteration)
run to the stop rule (relative change of u1, tolerance 1e-8 with the
a-posteriori bound) for each of the three delta values, followed by the flow
rate Q.  Inputs (geometry tables) are resident on the GPU before timing.

Reported: fluid-cell x velocity updates per second over the timed steps,
time to the converged flow rate per delta, the roofline of the dominant
kernel (the sweep) measured with HIP events on the solver's stream, and the
CPU oracle timed on the host on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("cell×velocity updates/s + % HBM peak; "
          "time-to-converged flow rate (1e-6) vs plain FP64")
DELTAS = (0.1, 1.0, 10.0)
NV = 64
TOL = 1e-8
FP64_VALU_PEAK = 78.6e12          # MI355X FP64 vector FLOP/s
# arithmetic the sweep performs per fluid cell x velocity update (FMA = 2):
# collision gain 3 FMA, upwind terms 2 x 2 FMA, combination 2 FMA,
# reciprocal-diagonal scaling 1 MUL, quadrature moments 1 MUL + 1 ADD + 3 FMA
FLOPS_PER_UPDATE = 6 + 8 + 4 + 1 + 8


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--precision", choices=["fp64", "fp32_refine"], default="fp64",
                   help="fp64 sweeps, or FP32 sweeps with FP64 defect correction")
    p.add_argument("--cpu-seconds", type=float, default=15.0,
                   help="budget of the CPU-oracle baseline sample")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--workload", choices=["rough_channel", "batch64", "couette", "porous", "adjoint"], default="rough_channel",
                   help="rough_channel: the headline workload; batch64: 64 uneven instances "
                        "(sides 64-384, 48 x 48 velocities) in one batched solve, throughput over a "
                        "fixed number of iterations; couette: the Couette flow of the fractal rough "
                        "channel and the smooth one over Kn 0.03-10 (Q*); porous: the rarefaction "
                        "sweep of the 512 x 512 porous cell (8 deltas over 0.01-100, warm starts) "
                        "and its permeability post-processing; adjoint: forward solve and gradient "
                        "of the 256 x 256 porous cell with delta(x) and alpha 0.9")
    p.add_argument("--batch-iters", type=int, default=24,
                   help="iterations per timed batched solve (batch64); 0: every instance "
                        "to the stop rule")
    p.add_argument("--schedule", choices=["auto", "skew", "wrap"], default="auto",
                   help="sweep order: auto (wrap-around diagonal, skewed order for instances "
                        "that stop contracting), skew (lags periodic/strip seams only) or "
                        "wrap (fewer steps, not unconditionally stable)")
    p.add_argument("--accel", choices=["auto", "none", "gmres"], default="auto",
                   help="auto: source iteration with extrapolation of its dominant mode, GMRES for "
                        "an instance that stops contracting; none: plain source iteration (the "
                        "paper's); gmres: GMRES on its fixed-point map")
    p.add_argument("--tol", type=float, default=TOL,
                   help="stop-rule tolerance of every solve (relative change of u1 and its "
                        "a-posteriori error bound)")
    p.add_argument("--block-iters", type=int, default=32,
                   help="iterations per captured block (the stop and rate checks run between blocks)")
    p.add_argument("--vel", type=int, default=0)
    p.add_argument("--waves", type=int, default=0)
    p.add_argument("--no-roofline", action="store_true",
                   help="skip the event-timed roofline pass (for profiler runs)")
    p.add_argument("--copy-calibration-mib", type=int, default=0,
                   help="first run a plain device copy of this many MiB (the "
                        "reference for profiler byte counters)")
    p.add_argument("--traffic-json", default=None,
                   help="HBM bytes per sweep launch measured by a profiler "
                        "(JSON {fetch_bytes, write_bytes}) to report as traffic")
    return p.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; "
                          "the solver has no multi-GPU path", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU available"}))
        sys.exit(1)
    import paper_1704_03126_amd.dvm as dvm
    from paper_1704_03126_amd.geometry import cfg_rough_channel

    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.workload == "batch64":
        return bench_batch(args, torch, dvm)
    if args.workload == "couette":
        return bench_couette(args, torch, dvm)
    if args.workload == "porous":
        return bench_porous(args, torch, dvm)
    if args.workload == "adjoint":
        return bench_adjoint(args, torch, dvm)

    g = cfg_rough_channel()
    nf = g.n_fluid
    K = NV * NV
    prec = dvm.DVM_FP32_REFINE if args.precision == "fp32_refine" else dvm.DVM_FP64
    solver = dvm.Solver(NV, 1, tol=args.tol, vel_per_lane=args.vel, waves_per_block=args.waves,
                        precision=prec, **solver_options(args, dvm))
    solver.set_geometry(0, g.mask, g.periodic_y, g.cells_per_H)

    scheds = {}

    def step():
        its, Qs, tts = [], [], []
        for d in DELTAS:
            t0 = time.perf_counter()
            info = solver.solve(0, d)
            Q, _ = solver.flow_rate(0)
            tts.append(time.perf_counter() - t0)
            its.append(info.iters)
            Qs.append(Q)
            scheds[str(d)] = info.schedule
        return its, Qs, tts

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    all_its, all_tts = [], []
    for _ in range(args.steps):
        its, Qs, tts = step()
        all_its.append(its)
        all_tts.append(tts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    iters = int(np.sum(all_its))
    updates = float(iters) * nf * K
    value = updates / elapsed
    ms_per_step = 1e3 * elapsed / args.steps

    roofline = None
    if not args.no_roofline:
        # roofline of the sweep: one more step with every sweep bracketed by
        # HIP events on the solver's stream
        prof = dvm.Solver(NV, 1, tol=args.tol, profile=True, vel_per_lane=args.vel,
                          waves_per_block=args.waves, **solver_options(args, dvm))
        prof.set_geometry(0, g.mask, g.periodic_y, g.cells_per_H)
        prof_sched = set()
        prof_iters = 0
        for d in DELTAS:
            pinfo = prof.solve(0, d)
            prof_sched.add(pinfo.schedule)
            prof_iters += pinfo.iters
        sweep_ms, n_sweeps, other_ms = prof.profile()
        (pv, pg), _ = prof.launch_shape()
        prof.close()
        kernel_sched = prof_sched.pop() if len(prof_sched) == 1 else "mixed" 
        avg_sweep_s = sweep_ms / max(n_sweeps, 1) / 1e3
        flops_per_launch = float(nf) * K * FLOPS_PER_UPDATE
        achieved = flops_per_launch / avg_sweep_s
        traffic = None
        traffic_detail = None
        tr = None
        if args.traffic_json:
            with open(args.traffic_json) as f:
                tr = json.load(f)
        else:
            tr = measured_traffic(kernel_sched, pv, pg)
        if tr is not None:
            traffic = tr["fetch_bytes"] + tr["write_bytes"]
            traffic_detail = {"fetch_bytes_per_launch": tr["fetch_bytes"],
                              "write_bytes_per_launch": tr["write_bytes"],
                              "bytes_per_update": traffic / (nf * K),
                              "hbm_GBps_at_avg_launch": traffic / avg_sweep_s / 1e9,
                              "source": tr.get("source", "")}
        roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": FP64_VALU_PEAK / 1e12,
                    "unit": "TFLOP/s", "frac": achieved / FP64_VALU_PEAK, "traffic": traffic,
                    "traffic_detail": traffic_detail,
                    "kernel": f"k_sweep<double,{pv},{pg}> ({kernel_sched} order)",
                    "avg_launch_ms": avg_sweep_s * 1e3,
                    "flops_per_update": FLOPS_PER_UPDATE, "updates_per_launch": nf * K,
                    "launches_timed": n_sweeps, "iterations_timed": prof_iters,
                    "sweep_share_of_iteration": sweep_ms / max(sweep_ms + other_ms, 1e-30)}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(g, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "rough_channel_256x128_blocks26x128_nv64_delta0.1_1_10",
                   "nx": g.nx, "ny": g.ny, "fluid_cells": nf, "velocities": K,
                   "deltas": list(DELTAS), "tol": args.tol, "precision": args.precision,
                   "schedule": args.schedule, "accel": args.accel, "block_iters": args.block_iters,
                   "parallelism": "single_gpu"},
        "iterations_per_delta": all_its[-1],
        "schedule_per_delta": scheds,
        "time_to_solution_s": dict(zip([str(d) for d in DELTAS],
                                       np.mean(np.array(all_tts), axis=0).tolist())),
        "Q": dict(zip([str(d) for d in DELTAS], Qs)),
        "Q_rel_err_vs_stored_oracle": stored_oracle_error(g, Qs),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    solver.close()
    print(json.dumps(out))


def solver_options(args, dvm):
    """Sweep order, acceleration and iteration-block length chosen on the
    command line."""
    return {"schedule": {"auto": dvm.DVM_SCHED_AUTO, "skew": dvm.DVM_SCHED_SKEW,
                         "wrap": dvm.DVM_SCHED_WRAP}[args.schedule],
            "accel": {"auto": dvm.DVM_ACCEL_AUTO, "none": dvm.DVM_ACCEL_NONE,
                      "gmres": dvm.DVM_ACCEL_GMRES}[args.accel],
            "block_iters": args.block_iters}


def stored_oracle_error(g, Qs):
    """|Q - Q_oracle| / |Q_oracle| per delta against the stored FP64 oracle
    results of this geometry (solved to 1e-12 on the CPU and kept as JSON
    with the tests), or None where none are stored."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                        f"rough_channel_{g.nx}x{g.ny}_nv{NV}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        ref = {float(r["delta"]): r["Q"] for r in json.load(f)["results"]}
    return {str(d): (abs(q - ref[d]) / abs(ref[d]) if d in ref else None) for d, q in zip(DELTAS, Qs)}


def bench_batch(args, torch, dvm):
    """64 uneven instances (seeded rough channels and porous cells, sides
    64-384, delta log-uniform on [0.01, 100]), 48 x 48 velocities, all in one
    batched launch sequence; every timed solve runs a fixed number of
    iterations (instances converge at very different counts, so throughput
    over a fixed budget is the comparable figure), or, with --batch-iters 0,
    runs every instance to the stop rule (time to solution of the batch)."""
    from paper_1704_03126_amd.geometry import batch_instances
    nv = 48
    gs = batch_instances(64)
    deltas = [g.meta["delta"] for g in gs]
    prec = dvm.DVM_FP32_REFINE if args.precision == "fp32_refine" else dvm.DVM_FP64
    to_conv = args.batch_iters <= 0
    s = dvm.Solver(nv, len(gs), tol=args.tol, max_iter=100000 if to_conv else args.batch_iters,
                   vel_per_lane=args.vel or 4, waves_per_block=args.waves or 8, precision=prec,
                   **solver_options(args, dvm))
    for i, g in enumerate(gs):
        s.set_geometry(i, g.mask, g.periodic_y, g.cells_per_H)
    nfl = [g.n_fluid for g in gs]
    for _ in range(max(args.warmup, 1)):
        s.solve(-1, deltas, raise_on_noconv=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    updates = 0.0
    for _ in range(args.steps):
        infos = s.solve(-1, deltas, raise_on_noconv=False)
        updates += sum(inf.iters * n for inf, n in zip(infos, nfl)) * nv * nv
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    Qs = [s.flow_rate(i)[0] for i in range(len(gs))] if to_conv else None
    s.close()
    out = {"metric": METRIC, "value": updates / elapsed, "unit": "updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if prec == dvm.DVM_FP64 else "f32+f64", "data": "synthetic",
           "config": {"workload": "batch64_uneven_sides64-384_nv48", "instances": len(gs),
                      "cells": int(sum(g.nx * g.ny for g in gs)), "fluid_cells": int(sum(nfl)),
                      "velocities": nv * nv,
                      "iterations_per_solve": "to the stop rule" if to_conv else args.batch_iters,
                      "tol": args.tol if to_conv else None, "precision": args.precision,
                      "schedule": args.schedule, "accel": args.accel, "parallelism": "single_gpu"},
           "roofline": None, "cpu_baseline": None}
    if to_conv:
        out["iterations_per_instance"] = [inf.iters for inf in infos]
        out["status_per_instance"] = [inf.status for inf in infos]
        out["delta_per_instance"] = deltas
        out["Q"] = Qs
    print(json.dumps(out))


def bench_couette(args, torch, dvm):
    """Couette flow of Sec. II: the fractal (D = 1.5, eps = 2 %) rough channel
    of aspect ratio 5 on graded rows (60 across the rough band, 100 above it,
    64 columns per H) and the smooth channel, top plate sliding at
    U0/v_m = 1, 32 x 32 velocities, Kn 0.03-10; one step = every Kn for both
    channels, solved to tol 1e-8 (warm starts along the Kn list).  Reports
    Q_r, Q_s and Q* = Q_r / Q_s per Kn."""
    from paper_1704_03126_amd.geometry import graded_fractal_couette_channel, plane_channel
    nv = 32
    kns = [0.03, 0.1, 0.3, 1.0, 3.0, 10.0]
    deltas = [float(np.sqrt(np.pi) / (2 * kn)) for kn in kns]
    rough = graded_fractal_couette_channel(64, n_band=60, n_rest=100, aspect=5, D=1.5, eps=0.02)
    smooth = plane_channel(64, 1)
    solvers = []
    for g in (rough, smooth):
        s = dvm.Solver(nv, 1, tol=args.tol, precision=dvm.DVM_FP32_REFINE if args.precision == "fp32_refine"
                       else dvm.DVM_FP64, **solver_options(args, dvm))
        s.set_geometry(0, g.mask, g.periodic_y, g.cells_per_H)
        if "dy" in g.meta:
            s.set_row_heights(0, g.meta["dy"])
        s.set_driving(0, 0.0, (0.0, 1.0))
        solvers.append((s, g))

    def step():
        out, upd = [], 0.0
        for s, g in solvers:
            Qs, infos = s.delta_sweep(0, deltas[::-1])     # continuum end first: warm starts
            out.append(Qs[::-1])
            upd += sum(i.iters for i in infos) * g.n_fluid * nv * nv
        return out, upd

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    upd = 0.0
    for _ in range(args.steps):
        (qr, qs), u = step()
        upd += u
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for s, _ in solvers:
        s.close()
    out = {"metric": METRIC, "value": upd / elapsed, "unit": "updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if args.precision == "fp64" else "f32+f64", "data": "synthetic",
           "config": {"workload": "couette_wm_D1.5_eps0.02_aspect5_graded60+100rows_64perH_nv32",
                      "rough_cells": [rough.ny, rough.nx], "Kn": kns, "tol": args.tol,
                      "precision": args.precision, "schedule": args.schedule, "accel": args.accel,
                      "parallelism": "single_gpu"},
           "Q_rough": [float(q) for q in qr], "Q_smooth": [float(q) for q in qs],
           "Q_star": [float(a / b) for a, b in zip(qr, qs)],
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(out))


def bench_porous(args, torch, dvm):
    """Rarefaction sweep of the periodic porous cell (Sec. III): 512 x 512
    cells, seeded overlapping discs (radius 0.03-0.08 of the side) to
    porosity 0.6 with non-percolating pores filled, 64 x 64 velocities,
    delta log-spaced over [0.01, 100] (8 values), each solve warm-started
    from the previous one (rarefied end first).  Reports per-delta sweeps,
    time and Q, and the post-processing: k_inf, H*, Kn*, k_a/k_inf."""
    from paper_1704_03126_amd.geometry import cfg_porous
    nv = 64
    g = cfg_porous()
    deltas = [float(d) for d in np.logspace(-2, 2, 8)]
    phi = float(np.mean(g.mask == 0))
    s = dvm.Solver(nv, 1, tol=args.tol, precision=dvm.DVM_FP32_REFINE if args.precision == "fp32_refine"
                   else dvm.DVM_FP64, **solver_options(args, dvm))
    s.set_geometry(0, g.mask, g.periodic_y, g.cells_per_H)

    def step():
        Qs, its, tts = [], [], []
        for i, d in enumerate(deltas):
            t = time.perf_counter()
            info = s.solve(0, d, warm=i > 0)
            Qs.append(s.flow_rate(0)[0])
            torch.cuda.synchronize()
            tts.append(time.perf_counter() - t)
            if info.status != "converged":
                raise RuntimeError(f"delta {d}: {info.status}")
            its.append(info.iters)
        return Qs, its, tts

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    upd = 0.0
    for _ in range(args.steps):
        Qs, its, tts = step()
        upd += sum(its) * g.n_fluid * nv * nv
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s.close()
    perm = dvm.permeability(deltas, Qs, phi)
    out = {"metric": METRIC, "value": upd / elapsed, "unit": "updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if args.precision == "fp64" else "f32+f64", "data": "synthetic",
           "config": {"workload": "porous_discs_512x512_phi0.6_seed1003_nv64_delta0.01-100x8",
                      "nx": g.nx, "ny": g.ny, "fluid_cells": g.n_fluid, "porosity": phi,
                      "velocities": nv * nv, "deltas": deltas, "tol": args.tol,
                      "precision": args.precision, "schedule": args.schedule, "accel": args.accel,
                      "parallelism": "single_gpu"},
           "iterations_per_delta": its, "time_to_solution_s": tts, "Q": Qs,
           "k_inf": perm["k_inf"], "H_star": perm["H_star"],
           "Kn_star": [float(x) for x in perm["Kn_star"]],
           "ka_over_kinf": [float(x) for x in perm["ka_ratio"]],
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(out))


def bench_adjoint(args, torch, dvm):
    """The gradient workload: a 256 x 256 periodic porous cell (porosity
    0.55, seed 3005), log-normal delta(x) of mean 1 smoothed over 8 cells
    (seed 3006), accommodation 0.9, 48 x 48 velocities, FP64.  One step = the
    forward solve to the stop rule and the gradient (dQ/d delta per cell and
    dQ/d alpha: checkpoint sweep, adjoint solve, gradient sweep), timed
    apart."""
    from paper_1704_03126_amd.geometry import delta_field, porous_discs
    nv, alpha = 48, 0.9
    g = porous_discs(256, 0.55, 3005)
    base = np.where(g.mask == 0, delta_field(g.mask.shape, 3006), 0.0)
    s = dvm.Solver(nv, 1, tol=args.tol, **solver_options(args, dvm))
    s.set_geometry(0, g.mask, g.periodic_y, g.cells_per_H)

    def step():
        t0 = time.perf_counter()
        info = s.solve(0, base, alpha)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gd, ga = s.grad(0)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return info, gd, ga, t1 - t0, t2 - t1

    for _ in range(args.warmup):
        step()
    fwd, adj, its = [], [], 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info, gd, ga, tf, ta = step()
        fwd.append(tf)
        adj.append(ta)
        its += info.iters
    elapsed = time.perf_counter() - t0
    Q = s.flow_rate(0)[0]
    s.close()
    out = {"metric": METRIC, "value": its * g.n_fluid * nv * nv / sum(fwd), "unit": "updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "adjoint_porous_256x256_phi0.55_seed3005_deltafield_alpha0.9_nv48",
                      "nx": g.nx, "ny": g.ny, "fluid_cells": g.n_fluid, "velocities": nv * nv,
                      "alpha": alpha, "tol": args.tol, "schedule": args.schedule, "accel": args.accel,
                      "parallelism": "single_gpu"},
           "value_is": "forward-solve updates/s", "forward_iterations": info.iters,
           "forward_s": float(np.mean(fwd)), "gradient_s": float(np.mean(adj)),
           "gradient_over_forward": float(np.mean(adj) / np.mean(fwd)),
           "Q": Q, "dQ_dalpha": ga, "dQ_ddelta_max_abs": float(np.max(np.abs(gd))),
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(out))


def measured_traffic(schedule, vel, waves):
    """Profiler-measured HBM bytes per sweep launch (profiles/), valid only
    while the kernel source, the sweep order and the launch shape are the
    ones that were profiled."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_sweep_traffic.json")
    src = os.path.join(ROOT, "paper_1704_03126_amd", "csrc", "dvm_kernels.hip")
    if not (os.path.exists(path) and os.path.exists(src)):
        return None
    with open(path) as f:
        tr = json.load(f)
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if not sha.startswith(tr.get("kernel_source_sha256_prefix", "-")):
        return None
    if tr.get("schedule") != schedule or tr.get("shape") != [vel, waves]:
        return None
    return tr


def cpu_baseline(g, budget_s):
    """The CPU oracle (FP64 source iteration) on a bounded sample of the same
    workload: full geometry and velocity grid, a fixed number of iterations
    scaled to take about `budget_s` seconds."""
    import oracle
    oracle.build(force=False)

    def run(n):
        t0 = time.perf_counter()
        oracle.si_solve(g.mask, 1.0, NV, periodic_y=g.periodic_y, cells_per_H=g.cells_per_H,
                        tol=-1.0, max_iter=n)
        return time.perf_counter() - t0

    # per-iteration cost from the difference of two short runs (a call also
    # pays the oracle's set-up), then as many iterations as fill the budget
    t1, t3 = run(1), run(3)
    it_s = max((t3 - t1) / 2.0, 1e-3)
    n = max(2, int(max(budget_s - t1 + it_s, it_s) / it_s))
    t0 = time.perf_counter()
    oracle.si_solve(g.mask, 1.0, NV, periodic_y=g.periodic_y, cells_per_H=g.cells_per_H,
                    tol=-1.0, max_iter=n)
    dt = time.perf_counter() - t0
    ups = n * g.n_fluid * NV * NV / dt
    return {"value": ups, "unit": "updates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{n} source iterations of the full workload at delta=1 "
                      f"({g.nx}x{g.ny} cells, {NV}x{NV} velocities), {dt:.1f} s"}


if __name__ == "__main__":
    main()
