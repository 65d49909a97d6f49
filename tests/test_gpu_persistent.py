"""Blocks of source iterations as one cooperative launch (persistent = 1)
against the same blocks as separate launches replayed from HIP graphs.

Every phase of the cooperative kernel computes what its separate kernel
computes, in the same order: the sweep's work items (taken from a device
counter instead of the launch grid), the moments (four lanes per cell, the
quadrant sums combined in the same order), the FP32 correction's add, the
records and the stop rule (max-reductions, order independent).  So the two
paths agree bit for bit: iteration counts, stop states, flow rates and
fields.  The oracle parity of these batches is covered by the batch tests.
"""
import numpy as np
import pytest

from paper_1704_03126_amd.geometry import batch_instances, rough_channel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dvm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1704_03126_amd.dvm as d
    d.load_library()
    return d


def _solve(dvm, gs, deltas, nv, persistent, precision, accel, tol=1e-10, rows=None):
    s = dvm.Solver(nv, len(gs), tol=tol, precision=precision, accel=accel, persistent=persistent,
                   vel_per_lane=4, waves_per_block=8)
    for i, g in enumerate(gs):
        s.set_geometry(i, g.mask, g.periodic_y, g.cells_per_H)
    if rows is not None:
        s.set_row_heights(0, rows)
    infos = s.solve(-1, deltas)
    out = [(s.flow_rate(i)[0], s.moments(i)) for i in range(len(gs))]
    prof = s.profile()
    s.close()
    return infos, out, prof


def _same(a, b):
    (ia, oa, _), (ib, ob, _) = a, b
    for x, y in zip(ia, ib):
        assert (x.status, x.iters, x.sweeps_fp64) == (y.status, y.iters, y.sweeps_fp64), (x, y)
        assert x.rel_change == y.rel_change
    for (qa, ma), (qb, mb) in zip(oa, ob):
        assert qa == qb
        for k in ma:
            assert np.array_equal(ma[k], mb[k]), k


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
@pytest.mark.parametrize("accel", ["none", "auto"])
def test_uneven_batch_bitwise(dvm, precision, accel):
    gs = batch_instances(6, seed=2024, smin=24, smax=96)
    rng = np.random.default_rng(11)
    deltas = [float(10.0 ** rng.uniform(-1.0, 1.0)) for _ in gs]
    prec = dvm.DVM_FP32_REFINE if precision == "fp32_refine" else dvm.DVM_FP64
    acc = dvm.DVM_ACCEL_NONE if accel == "none" else dvm.DVM_ACCEL_AUTO
    print(f"[persistent] batch of {len(gs)} nv=24 {precision} accel={accel}", flush=True)
    ref = _solve(dvm, gs, deltas, 24, False, prec, acc)
    got = _solve(dvm, gs, deltas, 24, True, prec, acc)
    assert ref[2]["persistent_blocks"] == 0
    assert got[2]["persistent_blocks"] > 0 and got[2]["persistent_iters"] >= got[2]["persistent_blocks"]
    assert all(inf.status == "converged" for inf in got[0])
    assert len({inf.iters for inf in got[0]}) > 1        # instances stopped on their own
    _same(ref, got)


def test_per_cell_delta_path_bitwise(dvm):
    """Rows of unequal height take the per-cell path of the sweep."""
    g = rough_channel(48, 32, 6, 24)
    dy = (1.0 / g.ny) * (1 + 0.8 * np.sin(np.linspace(0, 3, g.ny)) ** 2)
    print("[persistent] nonuniform rows 48x32 nv=16", flush=True)
    ref = _solve(dvm, [g], [1.0], 16, False, dvm.DVM_FP64, dvm.DVM_ACCEL_AUTO, rows=dy)
    got = _solve(dvm, [g], [1.0], 16, True, dvm.DVM_FP64, dvm.DVM_ACCEL_AUTO, rows=dy)
    assert got[2]["persistent_blocks"] > 0
    _same(ref, got)


def test_specular_walls_fall_back(dvm):
    """alpha < 1 needs the face buffers of the specular share: those blocks
    run as separate launches, with the same result."""
    g = rough_channel(40, 24, 5, 20)
    print("[persistent] specular fallback 40x24 nv=12", flush=True)
    res = []
    for persistent in (False, True):
        s = dvm.Solver(12, 1, tol=1e-10, persistent=persistent, vel_per_lane=4, waves_per_block=8)
        s.set_geometry(0, g.mask, g.periodic_y, g.cells_per_H)
        inf = s.solve(0, 1.0, 0.8)
        res.append((inf.iters, s.flow_rate(0)[0], s.profile()["persistent_blocks"]))
        s.close()
    assert res[0][:2] == res[1][:2]
    assert res[1][2] == 0
