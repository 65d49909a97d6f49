#!/usr/bin/env python3
"""Benchmark of the gfx950 linearized-BGK DVM solver (one JSON line).

Default workload: the uneven batch -- 64 independent instances (seeded
periodic porous cells and rough channels, sides 64-384 cells, delta
log-uniform on [0.01, 100]), 48 x 48 velocities of Eq. (nonuniform_v), all
in one context and one batched launch sequence, solved by FP32 sweeps with
FP64 moments and FP64 defect correction.  One step = one batched solve of
every instance from zero for a fixed budget of source iterations (32 by
default: a captured block of Eq. (iteration)), followed by the flow rate Q
of Sec. III of every instance.  Inputs (geometry tables) are resident on the
GPU before timing.

Reported on one line:
* value: fluid-cell x velocity updates per second over the timed steps (FP32
  and FP64 sweeps counted alike);
* roofline: algorithmic HBM bytes of the dominant kernel (the FP32 sweep:
  4 bytes per update -- one FP32 state element per fluid cell and velocity)
  over its average launch time, measured with HIP events on the solver's
  stream during the timed steps, against 8 TB/s; the FP64 sweeps of the
  same steps (8 bytes per update) and the profiler-measured bytes alongside;
* time to the converged flow rate (tol 1e-6) of the whole batch for FP32 +
  refinement and for the FP64 solver, each once after the timed steps, with
  Q's distance from the stored FP64 oracle results of four instances;
* cpu_baseline: the FP64 CPU oracle on a bounded sample of the same batch
  (all host cores, and one core).

Other workloads (--workload): rough_channel, couette, porous, adjoint.
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
HBM_PEAK = 8.0e12                 # MI355X HBM3E bytes/s
FP64_VALU_PEAK = 78.6e12          # MI355X FP64 vector FLOP/s
VALU_SIMDS = 256 * 4               # MI355X: 256 CUs x 4 SIMDs
CLOCK_HZ = 2.4e9                   # MI355X peak engine clock
# arithmetic the sweep performs per fluid cell x velocity update (FMA = 2):
# collision gain 3 FMA, upwind terms 2 x 2 FMA, combination 2 FMA,
# reciprocal-diagonal scaling 1 MUL, quadrature moments 1 MUL + 1 ADD + 3 FMA
FLOPS_PER_UPDATE = 6 + 8 + 4 + 1 + 8
# algorithmic HBM bytes per fluid cell x velocity update of a sweep that
# produces one state element per update and fuses the moments: the element
# itself, 8 bytes in FP64 and 4 in FP32 (the moments, records and lagged
# values add well under a byte per update)
BYTES_PER_UPDATE = {"fp64": 8, "fp32": 4}
BATCH_NV = 48
BATCH_TTS_TOL = 1e-6


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--precision", choices=["fp64", "fp32_refine"], default=None,
                   help="fp64 sweeps, or FP32 sweeps with FP64 defect correction (default: "
                        "fp32_refine for batch64, fp64 for the other workloads)")
    p.add_argument("--cpu-seconds", type=float, default=15.0,
                   help="budget of the CPU-oracle baseline sample")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--workload", choices=["rough_channel", "batch64", "couette", "porous", "adjoint"], default="batch64",
                   help="batch64 (default): 64 uneven instances (sides 64-384, 48 x 48 velocities) "
                        "in one batched solve, throughput over a fixed number of iterations per step "
                        "and time to solution of the batch; rough_channel: the 256 x 128 rough channel "
                        "at delta 0.1, 1, 10 to the stop rule; couette: the Couette flow of the fractal rough "
                        "channel and the smooth one over Kn 0.03-10 (Q*); porous: the rarefaction "
                        "sweep of the 512 x 512 porous cell (8 deltas over 0.01-100, warm starts) "
                        "and its permeability post-processing; adjoint: forward solve and gradient "
                        "of the 256 x 256 porous cell with delta(x) and alpha 0.9")
    p.add_argument("--batch-iters", type=int, default=32,
                   help="iterations per timed batched solve (batch64); 0: every instance "
                        "to the stop rule")
    p.add_argument("--no-tts", action="store_true",
                   help="batch64: skip the time-to-solution runs (for profiler runs)")
    p.add_argument("--tts-solvers", default="fp32_refine,fp64,fp64_plain_iteration",
                   help="batch64: which time-to-solution runs to make (comma list of fp32_refine, "
                        "fp64, fp64_plain_iteration; for profiler runs)")
    p.add_argument("--tts-tol", type=float, default=BATCH_TTS_TOL,
                   help="batch64: stop-rule tolerance of the time-to-solution runs")
    p.add_argument("--schedule", choices=["auto", "skew", "wrap"], default="auto",
                   help="sweep order: auto (wrap-around diagonal, skewed order for instances "
                        "that stop contracting), skew (lags periodic/strip seams only) or "
                        "wrap (fewer steps, not unconditionally stable)")
    p.add_argument("--accel", choices=["auto", "none", "gmres"], default="auto",
                   help="auto: source iteration with extrapolation of its dominant mode, GMRES for "
                        "an instance that stops contracting; none: plain source iteration (the "
                        "paper's); gmres: GMRES on its fixed-point map")
    p.add_argument("--tol", type=float, default=None,
                   help="stop-rule tolerance of every solve (relative change of u1 and its "
                        "a-posteriori error bound)")
    p.add_argument("--block-iters", type=int, default=32,
                   help="iterations per captured block (the stop and rate checks run between blocks)")
    p.add_argument("--alpha", type=float, default=0.9,
                   help="accommodation coefficient of the gradient workload (adjoint)")
    p.add_argument("--persistent", action="store_true",
                   help="run blocks of iterations as one cooperative launch (untimed sweeps only: "
                        "the roofline's timed steps use separate launches)")
    p.add_argument("--krylov-dim", type=int, default=0,
                   help="GMRES restart length (0: the library's default, 40 with deflated restarts)")
    p.add_argument("--krylov-deflate", type=int, default=0,
                   help="harmonic Ritz vectors a GMRES cycle hands to the next (0: the library's "
                        "default, negative: plain restarts)")
    p.add_argument("--continuation", action="store_true",
                   help="porous: warm starts from the state extrapolated in log(delta) through the "
                        "last two solutions (warm_extrapolate) instead of the last solution as it is")
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
    if args.precision is None:
        args.precision = "fp32_refine" if args.workload == "batch64" else "fp64"
    if args.tol is None:
        args.tol = TOL
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
        # HIP events on the solver's stream, in the same precision
        prof = dvm.Solver(NV, 1, tol=args.tol, profile=True, vel_per_lane=args.vel,
                          waves_per_block=args.waves, precision=prec, **solver_options(args, dvm))
        prof.set_geometry(0, g.mask, g.periodic_y, g.cells_per_H)
        prof_sched = set()
        prof_iters = 0
        for d in DELTAS:
            pinfo = prof.solve(0, d)
            prof_sched.add(pinfo.schedule)
            prof_iters += pinfo.iters
        p = prof.profile()
        (pv, pg), (pv32, pg32) = prof.launch_shape()
        prof.close()
        kernel_sched = prof_sched.pop() if len(prof_sched) == 1 else "mixed"
        f32 = p["n_sweeps32"] > 0 and p["sweep32_ms"] >= p["sweep_ms"]
        leg = "fp32" if f32 else "fp64"
        ms, n, upd = ((p["sweep32_ms"], p["n_sweeps32"], p["updates32"]) if f32
                      else (p["sweep_ms"], p["n_sweeps"], p["updates"]))
        avg_sweep_s = ms / max(n, 1) / 1e3
        bytes_per_launch = BYTES_PER_UPDATE[leg] * upd / max(n, 1)
        achieved = bytes_per_launch / avg_sweep_s
        traffic = None
        traffic_detail = None
        if args.traffic_json:
            with open(args.traffic_json) as f:
                tr = json.load(f)
        else:
            tr = measured_traffic("rough_channel", leg, pv32 if f32 else pv, pg32 if f32 else pg,
                                  schedule=kernel_sched)
        if tr is not None:
            traffic = tr["fetch_bytes"] + tr["write_bytes"]
            traffic_detail = {"fetch_bytes_per_launch": tr["fetch_bytes"],
                              "write_bytes_per_launch": tr["write_bytes"],
                              "measured_over_algorithmic": traffic / bytes_per_launch,
                              "source": tr.get("source", "")}
        flops = float(upd / max(n, 1)) * FLOPS_PER_UPDATE / avg_sweep_s
        roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK, "traffic": traffic,
                    "traffic_detail": traffic_detail,
                    "kernel": (f"k_sweep<{'float' if f32 else 'double'},{pv32 if f32 else pv},"
                               f"{pg32 if f32 else pg}> ({kernel_sched} order)"),
                    "avg_launch_ms": avg_sweep_s * 1e3, "bytes_per_update": BYTES_PER_UPDATE[leg],
                    "updates_per_launch": upd / max(n, 1), "launches_timed": n,
                    "iterations_timed": prof_iters,
                    "valu": {"flops_per_update": FLOPS_PER_UPDATE, "achieved_TFLOPs": flops / 1e12,
                             "frac_of_fp64_vector_peak": flops / FP64_VALU_PEAK},
                    "sweep_share_of_iteration": p["sweep_ms"] / max(p["sweep_ms"] + p["other_ms"], 1e-30)}

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
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "rough_channel_256x128_blocks26x128_nv64_delta0.1_1_10",
                   "nx": g.nx, "ny": g.ny, "fluid_cells": nf, "velocities": K,
                   "deltas": list(DELTAS), "tol": args.tol, "precision": args.precision,
                   "schedule": args.schedule, "accel": args.accel, "krylov": krylov_config(args), "block_iters": args.block_iters,
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
            "block_iters": args.block_iters, "persistent": args.persistent,
            "krylov_dim": args.krylov_dim, "krylov_deflate": args.krylov_deflate}


def krylov_config(args):
    """GMRES restart length and kept harmonic Ritz vectors as the library
    applies them (0 selects its defaults: 40 and 10 with deflated restarts,
    64 with plain ones)."""
    deflate = args.krylov_deflate >= 0
    m = args.krylov_dim if args.krylov_dim > 0 else (40 if deflate else 64)
    m = min(m, 64)
    kept = 0 if not deflate else min(args.krylov_deflate if args.krylov_deflate > 0 else m // 4, m // 2 - 1)
    return {"restart": m, "kept": max(kept, 0)}


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
    """The uneven batch: 64 seeded instances (even i: s x s porous cell of
    porosity 0.6; odd i: s x s/2 rough channel; s uniform on 64..384; delta
    log-uniform on [0.01, 100]), 48 x 48 velocities, one context, one
    batched launch sequence.  A step solves every instance from zero for
    --batch-iters source iterations (FP32 correction sweeps and FP64 steps
    of the refinement alike) and reads every Q; with --batch-iters 0 a step
    runs every instance to the stop rule."""
    from paper_1704_03126_amd.geometry import batch_instances
    nv = BATCH_NV
    K = nv * nv
    gs = batch_instances(64)
    deltas = [g.meta["delta"] for g in gs]
    nfl = [g.n_fluid for g in gs]
    prec = dvm.DVM_FP32_REFINE if args.precision == "fp32_refine" else dvm.DVM_FP64
    to_conv = args.batch_iters <= 0
    vel, waves = args.vel or 4, args.waves or 8
    prof_on = not args.no_roofline
    s = dvm.Solver(nv, len(gs), tol=args.tol, max_iter=200000 if to_conv else args.batch_iters,
                   vel_per_lane=vel, waves_per_block=waves, precision=prec, profile=prof_on,
                   **solver_options(args, dvm))
    for i, g in enumerate(gs):
        s.set_geometry(i, g.mask, g.periodic_y, g.cells_per_H)

    def step():
        infos = s.solve(-1, deltas, raise_on_noconv=False)
        Qs = [s.flow_rate(i)[0] for i in range(len(gs))]
        return infos, Qs

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    if prof_on:
        s.profile()                       # timings of the timed steps only
    t0 = time.perf_counter()
    updates, sweeps32, sweeps64 = 0.0, 0, 0
    for _ in range(args.steps):
        infos, Qs = step()
        updates += sum(inf.iters * n for inf, n in zip(infos, nfl)) * K
        sweeps64 += sum(inf.sweeps_fp64 for inf in infos)
        sweeps32 += sum(inf.iters - inf.sweeps_fp64 for inf in infos)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = s.profile() if prof_on else None
    s.close()

    roofline = batch_roofline(prof, vel, waves, args) if prof else None
    tts = None if args.no_tts else batch_time_to_solution(args, torch, dvm, gs, deltas, vel, waves)
    cpu = None if args.no_cpu else cpu_baseline_batch(gs, nv, args.cpu_seconds)
    prec_name = "fp32_refine" if prec == dvm.DVM_FP32_REFINE else "fp64"
    out = {"metric": METRIC, "value": updates / elapsed, "unit": "updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if prec == dvm.DVM_FP64 else "f32+f64",
           "data": "synthetic",
           "config": {"workload": "batch64_uneven_porous+rough_sides64-384_delta0.01-100_nv48",
                      "instances": len(gs), "cells": int(sum(g.nx * g.ny for g in gs)),
                      "fluid_cells": int(sum(nfl)), "velocities": K,
                      "iterations_per_step": "to the stop rule" if to_conv else args.batch_iters,
                      "tol": args.tol if to_conv else None, "precision": prec_name,
                      "launch_shape": [vel, waves], "schedule": args.schedule, "accel": args.accel, "krylov": krylov_config(args),
                      "parallelism": "single_gpu"},
           "sweeps_per_step": {"fp32": sweeps32 // max(args.steps, 1), "fp64": sweeps64 // max(args.steps, 1)},
           "roofline": roofline, "time_to_solution": tts, "cpu_baseline": cpu}
    if to_conv:
        out["iterations_per_instance"] = [inf.iters for inf in infos]
        out["status_per_instance"] = [inf.status for inf in infos]
        out["Q_rel_err_vs_stored_oracle"] = batch_oracle_error(Qs)
    print(json.dumps(out))


def batch_roofline(prof, vel, waves, args):
    """Roofline of the dominant kernel of the timed steps: the sweep (FP32 in
    the refinement, else FP64), algorithmic bytes (BYTES_PER_UPDATE x fluid
    updates of the timed launches) over the launches' total event time."""
    legs = {}
    for name, ms, n, upd in (("fp64", prof["sweep_ms"], prof["n_sweeps"], prof["updates"]),
                             ("fp32", prof["sweep32_ms"], prof["n_sweeps32"], prof["updates32"])):
        if n == 0 or ms <= 0:
            continue
        t = ms / 1e3
        bpl = BYTES_PER_UPDATE[name] * upd / n
        legs[name] = {"launches": n, "avg_launch_ms": ms / n, "updates": upd,
                      "algorithmic_bytes_per_launch": bpl,
                      "achieved_GBps": BYTES_PER_UPDATE[name] * upd / t / 1e9,
                      "updates_per_s": upd / t, "time_ms": ms}
    if not legs:
        return None
    dom = max(legs, key=lambda k: legs[k]["time_ms"])
    d = legs[dom]
    tr = measured_traffic("batch64", dom, vel, waves)
    traffic = None
    detail = None
    valu = None
    if tr is not None:
        traffic = tr["fetch_bytes"] + tr["write_bytes"]
        detail = {"fetch_bytes_per_launch": tr["fetch_bytes"], "write_bytes_per_launch": tr["write_bytes"],
                  "measured_over_algorithmic": traffic / d["algorithmic_bytes_per_launch"],
                  "source": tr.get("source", "")}
        if tr.get("sq_insts_valu_per_launch"):
            # VALU issue: a wave64 VALU instruction holds a 16-lane SIMD for
            # 4 cycles; the profiled instruction count against the SIMD
            # cycles of this run's average launch
            cycles = VALU_SIMDS * CLOCK_HZ * d["avg_launch_ms"] / 1e3
            busy = 4.0 * tr["sq_insts_valu_per_launch"] / cycles
            valu = {"insts_per_launch": tr["sq_insts_valu_per_launch"], "simd_cycles_per_launch": cycles,
                    "issue_busy": busy, "source": "SQ_INSTS_VALU of the profiled run (profiles/)"}
    return {"bound": "hbm", "achieved": d["achieved_GBps"], "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": d["achieved_GBps"] * 1e9 / HBM_PEAK, "traffic": traffic, "traffic_detail": detail,
            "valu": valu, "kernel": f"k_sweep<{'float' if dom == 'fp32' else 'double'},{vel},{waves}>",
            "bytes_per_update": BYTES_PER_UPDATE[dom], "legs": legs,
            "timing": "HIP events around every sweep launch on the solver's stream, timed steps only"}


def batch_oracle_error(Qs):
    """|Q - Q_oracle| / |Q_oracle| for the instances with stored FP64 oracle
    results (tests/golden/batch64_subset_nv48.json, solved to 1e-12)."""
    path = os.path.join(ROOT, "tests", "golden", "batch64_subset_nv48.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        ref = json.load(f)
    return {str(r["index"]): abs(Qs[r["index"]] - r["Q"]) / abs(r["Q"]) for r in ref["instances"]}


def batch_time_to_solution(args, torch, dvm, gs, deltas, vel, waves):
    """Time to the converged flow rate of the whole batch at --tts-tol: FP32
    sweeps with FP64 refinement against the FP64 solver (AUTO acceleration
    both, and the FP64 plain source iteration), each once, with Q's error
    against the stored oracle results and between the two precisions."""
    runs = {}
    Qref = None
    for name, prec, accel in (("fp32_refine", dvm.DVM_FP32_REFINE, dvm.DVM_ACCEL_AUTO),
                              ("fp64", dvm.DVM_FP64, dvm.DVM_ACCEL_AUTO),
                              ("fp64_plain_iteration", dvm.DVM_FP64, dvm.DVM_ACCEL_NONE)):
        if name not in args.tts_solvers.split(","):
            continue
        s = dvm.Solver(BATCH_NV, len(gs), tol=args.tts_tol, max_iter=200000, precision=prec, accel=accel,
                       vel_per_lane=vel, waves_per_block=waves, block_iters=args.block_iters,
                       persistent=args.persistent, krylov_dim=args.krylov_dim,
                       krylov_deflate=args.krylov_deflate)
        for i, g in enumerate(gs):
            s.set_geometry(i, g.mask, g.periodic_y, g.cells_per_H)
        s.solve(1, deltas[1])             # layout, buffers and captured blocks, outside the timing
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = s.solve(-1, deltas, raise_on_noconv=False)
        Qs = [s.flow_rate(i)[0] for i in range(len(gs))]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s.close()
        conv = [inf.status == "converged" for inf in infos]
        r = {"seconds": dt, "converged": int(sum(conv)), "status": [inf.status for inf in infos],
             "sweeps_total": int(sum(inf.iters for inf in infos)),
             "sweeps_fp64_total": int(sum(inf.sweeps_fp64 for inf in infos)),
             "sweeps_max": int(max(inf.iters for inf in infos)),
             "Q_rel_err_vs_stored_oracle": batch_oracle_error(Qs)}
        if name == "fp32_refine":
            Qref = Qs
        elif Qref is not None:
            r["max_rel_Q_diff_vs_fp32_refine"] = max(
                abs(a - b) / abs(b) for a, b, ok in zip(Qref, Qs, conv) if ok)
        runs[name] = r
    runs["tol"] = args.tts_tol
    if "fp64" in runs and "fp32_refine" in runs:
        runs["speedup_fp32_refine_vs_fp64"] = runs["fp64"]["seconds"] / runs["fp32_refine"]["seconds"]
    return runs


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
                      "precision": args.precision, "schedule": args.schedule, "accel": args.accel, "krylov": krylov_config(args),
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
    from the previous one (rarefied end first; with --continuation from the
    third delta on from the state extrapolated in log(delta)).
    Reports per-delta sweeps,
    time and Q, and the post-processing: k_inf, H*, Kn*, k_a/k_inf."""
    from paper_1704_03126_amd.geometry import cfg_porous
    nv = 64
    g = cfg_porous()
    deltas = [float(d) for d in np.logspace(-2, 2, 8)]
    phi = float(np.mean(g.mask == 0))
    s = dvm.Solver(nv, 1, tol=args.tol, precision=dvm.DVM_FP32_REFINE if args.precision == "fp32_refine"
                   else dvm.DVM_FP64, warm_extrapolate=args.continuation, **solver_options(args, dvm))
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
                      "precision": args.precision, "schedule": args.schedule, "accel": args.accel, "krylov": krylov_config(args),
                      "continuation": args.continuation, "parallelism": "single_gpu"},
           "iterations_per_delta": its, "time_to_solution_s": tts, "Q": Qs,
           "k_inf": perm["k_inf"], "H_star": perm["H_star"],
           "Kn_star": [float(x) for x in perm["Kn_star"]],
           "ka_over_kinf": [float(x) for x in perm["ka_ratio"]],
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(out))


def bench_adjoint(args, torch, dvm):
    """The gradient workload: a 256 x 256 periodic porous cell (porosity
    0.55, seed 3005), log-normal delta(x) of mean 1 smoothed over 8 cells
    (seed 3006), accommodation --alpha (default 0.9), 48 x 48 velocities,
    FP64.  One step = the
    forward solve to the stop rule and the gradient (dQ/d delta per cell and
    dQ/d alpha: checkpoint sweep, adjoint solve, gradient sweep), timed
    apart."""
    from paper_1704_03126_amd.geometry import delta_field, porous_discs
    nv, alpha = 48, args.alpha
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
           "config": {"workload": f"adjoint_porous_256x256_phi0.55_seed3005_deltafield_alpha{alpha:g}_nv48",
                      "nx": g.nx, "ny": g.ny, "fluid_cells": g.n_fluid, "velocities": nv * nv,
                      "alpha": alpha, "tol": args.tol, "schedule": args.schedule, "accel": args.accel, "krylov": krylov_config(args),
                      "parallelism": "single_gpu"},
           "value_is": "forward-solve updates/s", "forward_iterations": info.iters,
           "forward_s": float(np.mean(fwd)), "gradient_s": float(np.mean(adj)),
           "gradient_over_forward": float(np.mean(adj) / np.mean(fwd)),
           "Q": Q, "dQ_dalpha": ga, "dQ_ddelta_max_abs": float(np.max(np.abs(gd))),
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(out))


KERNEL_SOURCES = ("dvm_kernels.hip", "dvm_sweep_body.inc", "dvm_internal.h")


def kernel_source_sha256():
    """sha256 over the sweep kernel's source files, in a fixed order (None if
    one is missing)."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        src = os.path.join(ROOT, "paper_1704_03126_amd", "csrc", name)
        if not os.path.exists(src):
            return None
        with open(src, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload, precision, vel, waves, schedule=None):
    """Profiler-measured HBM bytes per sweep launch (profiles/), valid only
    while the kernel source, the workload, the sweep precision, order and
    launch shape are the ones that were profiled."""
    path = os.path.join(ROOT, "profiles", "k_sweep_traffic.json")
    sha = kernel_source_sha256()
    if not (os.path.exists(path) and sha):
        return None
    with open(path) as f:
        entries = json.load(f)
    if isinstance(entries, dict):
        entries = [entries]
    for tr in entries:
        if not sha.startswith(tr.get("kernel_source_sha256_prefix", "-")):
            continue
        if tr.get("workload_key", "rough_channel") != workload:
            continue
        if tr.get("precision", "fp64") != precision or tr.get("shape") != [vel, waves]:
            continue
        if schedule is not None and tr.get("schedule") != schedule:
            continue
        return tr
    return None


def cpu_baseline_batch(gs, nv, budget_s):
    """The CPU oracle (FP64 source iteration, OpenMP over velocities) on a
    bounded sample of the batch: a fixed number of iterations of its largest
    instance on every host core, and of a small instance on one core, each
    scaled to about half of `budget_s`."""
    import oracle
    oracle.build(force=False)

    def timed(g, n):
        t0 = time.perf_counter()
        oracle.si_solve(g.mask, g.meta["delta"], nv, periodic_y=g.periodic_y, cells_per_H=g.cells_per_H,
                        tol=-1.0, max_iter=n)
        return time.perf_counter() - t0

    def sample(i, budget):
        g = gs[i]
        t1, t3 = timed(g, 1), timed(g, 3)
        it_s = max((t3 - t1) / 2.0, 1e-4)
        n = max(2, int(max(budget - t1 + it_s, it_s) / it_s))
        dt = timed(g, n)
        return n * g.n_fluid * nv * nv / dt, n, dt, g

    cores = oracle.num_threads()
    big = max(range(len(gs)), key=lambda i: gs[i].n_fluid)
    small = min(range(len(gs)), key=lambda i: gs[i].n_fluid)
    ups, n, dt, g = sample(big, 0.5 * budget_s)
    oracle.set_num_threads(1)
    ups1, n1, dt1, g1 = sample(small, 0.5 * budget_s)
    oracle.set_num_threads(cores)
    return {"value": ups, "unit": "updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} source iterations of batch instance {big} ({g.nx}x{g.ny} cells, "
                      f"{g.n_fluid} fluid, delta {g.meta['delta']:.4g}, {nv}x{nv} velocities), {dt:.1f} s",
            "one_core": {"value": ups1, "unit": "updates/s", "cores": 1,
                         "sample": f"{n1} source iterations of batch instance {small} ({g1.nx}x{g1.ny} "
                                   f"cells, {g1.n_fluid} fluid), {dt1:.1f} s"}}


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
