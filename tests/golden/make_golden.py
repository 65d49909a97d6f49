"""Write the stored expected values of the full-size parity tests.

Calls only the FP64 CPU oracle (oracle/); nothing here comes from the GPU
path.  Each fixture records the configuration, the oracle's flow rate Q of
Sec. III, its iteration count and stop statistics, and u1 at a few seeded
cells for element checks.  Run from the repository root:

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
from paper_1704_03126_amd.geometry import (cfg_plane_channel, cfg_porous,  # noqa: E402
                                           cfg_rough_channel)

TOL = 1e-12

CASES = {
    # plane Poiseuille channel, 64 cells across H, 32 x 32 velocities, delta = 1
    "plane_channel_64_nv32": (cfg_plane_channel, 32, [1.0]),
    # rough channel 256 x 128, blocks 0.2H x half period, 64 x 64 velocities
    "rough_channel_256x128_nv64": (cfg_rough_channel, 64, [0.1, 1.0, 10.0]),
    # porous unit cell 512 x 512, porosity 0.6, 64 x 64 velocities
    "porous_512_nv64": (cfg_porous, 64, [1.0]),
}


def sample_cells(mask, n, seed):
    rng = np.random.default_rng(seed)
    fl = np.argwhere(mask == 0)
    pick = fl[rng.choice(len(fl), size=min(n, len(fl)), replace=False)]
    return [[int(y), int(x)] for y, x in pick]


def make(name):
    make_geom, nv, deltas = CASES[name]
    g = make_geom()
    cells = sample_cells(g.mask, 16, 7)
    out = {"name": name, "nx": g.nx, "ny": g.ny, "nv": nv, "periodic_y": bool(g.periodic_y),
           "cells_per_H": g.cells_per_H, "oracle_tol": TOL, "source": "oracle.si_solve (FP64 CPU)",
           "cells": cells, "results": []}
    for d in deltas:
        t0 = time.time()
        r = oracle.si_solve(g.mask, d, nv, periodic_y=g.periodic_y, cells_per_H=g.cells_per_H,
                            tol=TOL, max_iter=200000)
        out["results"].append({"delta": d, "Q": r.Q, "iters": int(r.iters), "rel_change": float(r.eps),
                               "u1": [float(r.u1[y, x]) for y, x in cells],
                               "u2": [float(r.u2[y, x]) for y, x in cells]})
        print(f"{name} delta={d}: Q={r.Q:.15g} iters={r.iters} ({time.time() - t0:.0f} s)", flush=True)
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(CASES)):
        make(n)
