"""Write the stored expected values of the full-size parity tests.

Calls only the FP64 CPU oracle (oracle/); nothing here comes from the GPU
path.  Each fixture records the configuration, the oracle's flow rate Q of
Sec. III, its iteration count and stop statistics, and the moments of
Sec. II.A (rho with zero fluid mean, u1, u2, tau, and the shear stress P12):

* ``<name>.json``: the configuration, Q per delta, and the moments at 16 (or
  64) seeded fluid cells;
* ``<name>_fields.npz`` (cases with ``fields=True``): the whole ny x nx
  fields, keyed ``d<i>_<moment>`` for the i-th delta of the case.

Run from the repository root (the oracle uses every host core unless
OMP_NUM_THREADS says otherwise):

    python tests/golden/make_golden.py [name ...]
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1704_03126_amd.geometry import (batch_instances, cfg_plane_channel,  # noqa: E402
                                           cfg_porous, cfg_rough_channel)

TOL = 1e-12
MOMENTS = ("rho", "u1", "u2", "tau", "p12")

# name -> (geometry maker, nv, deltas, whole fields stored, oracle tolerance)
CASES = {
    # plane Poiseuille channel, 64 cells across H, 32 x 32 velocities, delta = 1
    "plane_channel_64_nv32": (cfg_plane_channel, 32, [1.0], True, TOL),
    # rough channel 256 x 128, blocks 0.2H x half period, 64 x 64 velocities
    "rough_channel_256x128_nv64": (cfg_rough_channel, 64, [0.1, 1.0, 10.0], True, TOL),
    # porous unit cell 512 x 512, porosity 0.6, 64 x 64 velocities
    "porous_512_nv64": (cfg_porous, 64, [1.0], True, TOL),
    # the same disc recipe (porosity 0.6, seed 1003) on a 128 x 128 cell: the
    # rarefaction sweep's end points and middle, where the 512 x 512 oracle
    # solves would take hours on the host
    "porous_128_nv64": (lambda: cfg_porous(128), 64, [0.01, 1.0, 100.0], True, 1e-11),
}

# instances of the 64-instance uneven batch (48 x 48 velocities, each at its
# own delta): the largest porous cell, the largest rough channel, the
# smallest delta, and the largest delta among the porous cells below 150^2
BATCH_PICK = (14, 13, 39, 36)
BATCH_NAME = "batch64_subset_nv48"


def sample_cells(mask, n, seed):
    rng = np.random.default_rng(seed)
    fl = np.argwhere(mask == 0)
    pick = fl[rng.choice(len(fl), size=min(n, len(fl)), replace=False)]
    return [[int(y), int(x)] for y, x in pick]


def _solve(g, d, nv, tol):
    t0 = time.time()
    r = oracle.si_solve(g.mask, d, nv, periodic_y=g.periodic_y, cells_per_H=g.cells_per_H,
                        tol=tol, max_iter=400000)
    return r, time.time() - t0


def _record(r, d, cells):
    rec = {"delta": d, "Q": r.Q, "iters": int(r.iters), "rel_change": float(r.eps),
           "converged": bool(r.converged)}
    for m in MOMENTS:
        f = getattr(r, m)
        rec[m] = [float(f[y, x]) for y, x in cells]
        rec[m + "_max_abs"] = float(np.max(np.abs(f)))
    return rec


def make(name):
    make_geom, nv, deltas, fields, tol = CASES[name]
    g = make_geom()
    cells = sample_cells(g.mask, 16, 7)
    out = {"name": name, "nx": g.nx, "ny": g.ny, "nv": nv, "periodic_y": bool(g.periodic_y),
           "cells_per_H": g.cells_per_H, "oracle_tol": tol, "source": "oracle.si_solve (FP64 CPU)",
           "cells": cells, "results": [], "fields": f"{name}_fields.npz" if fields else None}
    arrays = {}
    for i, d in enumerate(deltas):
        r, dt = _solve(g, d, nv, tol)
        out["results"].append(_record(r, d, cells))
        if fields:
            for m in MOMENTS:
                arrays[f"d{i}_{m}"] = getattr(r, m)
        print(f"{name} delta={d}: Q={r.Q:.15g} iters={r.iters} converged={r.converged} "
              f"({dt:.0f} s)", flush=True)
    if fields:
        np.savez_compressed(os.path.join(HERE, f"{name}_fields.npz"), **arrays)
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=1)


def make_batch():
    gs = batch_instances(64)
    nv = 48
    out = {"name": BATCH_NAME, "nv": nv, "oracle_tol": TOL, "source": "oracle.si_solve (FP64 CPU)",
           "generator": "paper_1704_03126_amd.geometry.batch_instances(64)", "instances": []}
    for i in BATCH_PICK:
        g = gs[i]
        d = g.meta["delta"]
        cells = sample_cells(g.mask, 64, 100 + i)
        r, dt = _solve(g, d, nv, TOL)
        rec = _record(r, d, cells)
        rec.update({"index": i, "nx": g.nx, "ny": g.ny, "periodic_y": bool(g.periodic_y),
                    "cells_per_H": g.cells_per_H, "cells": cells})
        out["instances"].append(rec)
        print(f"{BATCH_NAME}[{i}] {g.nx}x{g.ny} delta={d:.6g}: Q={r.Q:.15g} iters={r.iters} "
              f"converged={r.converged} ({dt:.0f} s)", flush=True)
        with open(os.path.join(HERE, BATCH_NAME + ".json"), "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(CASES) + [BATCH_NAME]):
        if n == BATCH_NAME:
            make_batch()
        else:
            make(n)
