"""GPU (gfx950) solver vs the FP64 CPU oracle, through the C ABI.

Both sides converge to the fixed point of the same discrete problem; the
bar is the one the flow-rate study needs: Q within 1e-6 relative and the
velocity field within 1e-5 max-abs (FP64), checked here much tighter where
both solves run to 1e-12..1e-10.  The GPU iteration lags values across strip
boundaries and its wrap-around diagonal while the oracle lags only periodic
seams, so iteration counts differ; fixed points do not.
"""
import numpy as np
import pytest

import oracle
from paper_1704_03126_amd.geometry import (delta_field, plane_channel,
                                           porous_discs, rough_channel)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dvm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1704_03126_amd.dvm as d
    d.load_library()
    return d


def gpu_solve(dvm, g, delta, nv, tol=1e-11, alpha=1.0, vel=0, waves=0, graphs=True,
              shear=False, max_iter=200000, schedule=0):
    s = dvm.Solver(nv, 1, tol=tol, vel_per_lane=vel, waves_per_block=waves,
                   use_graphs=graphs, max_iter=max_iter, schedule=schedule)
    s.set_geometry(0, g.mask, g.periodic_y, g.cells_per_H)
    info = s.solve(0, delta, alpha)
    Q, ka = s.flow_rate(0)
    mom = s.moments(0, shear=shear)
    s.close()
    return Q, ka, mom, info


def oracle_solve(g, delta, nv, tol=1e-12):
    return oracle.si_solve(g.mask, delta, nv, periodic_y=g.periodic_y,
                           cells_per_H=g.cells_per_H, tol=tol)


def assert_parity(Qg, momg, ref, qtol=1e-9, utol=1e-9):
    fl = ref.u1 != 0
    assert abs(Qg - ref.Q) <= qtol * abs(ref.Q), (Qg, ref.Q)
    assert np.max(np.abs(momg["u1"] - ref.u1)) <= utol, np.max(np.abs(momg["u1"] - ref.u1))
    assert np.max(np.abs(momg["u2"] - ref.u2)) <= utol


def test_plane_channel_nx1(dvm):
    """x-invariant channel, 64 cells across H, 32x32 velocities, delta = 1."""
    g = plane_channel(64)
    ref = oracle_solve(g, 1.0, 32)
    Q, ka, mom, info = gpu_solve(dvm, g, 1.0, 32)
    assert info.status == "converged"
    assert_parity(Q, mom, ref)
    assert abs(ka - Q) < 1e-15
    assert np.max(np.abs(mom["rho"] - ref.rho)) < 1e-8
    assert np.max(np.abs(mom["tau"] - ref.tau)) < 1e-8


@pytest.mark.parametrize("delta", [0.1, 1.0, 10.0])
def test_rough_channel_reduced(dvm, delta):
    g = rough_channel(64, 32, 6, 32)
    ref = oracle_solve(g, delta, 16)
    Q, _, mom, info = gpu_solve(dvm, g, delta, 16)
    assert info.status == "converged"
    assert_parity(Q, mom, ref, qtol=1e-8, utol=1e-8)
    # mirror symmetry of the aligned blocks
    assert np.max(np.abs(mom["u1"] - mom["u1"][::-1])) < 1e-9


def test_porous_periodic(dvm):
    g = porous_discs(64, 0.6, 1003)
    ref = oracle_solve(g, 1.0, 12)
    Q, _, mom, info = gpu_solve(dvm, g, 1.0, 12)
    assert info.status == "converged"
    assert_parity(Q, mom, ref, qtol=1e-8, utol=1e-9)


def test_multi_strip_and_ragged_sizes(dvm):
    # 150 rows -> 3 strips; 37 columns (not a multiple of anything)
    g = rough_channel(37, 150, 30, 11)
    ref = oracle_solve(g, 0.7, 8)
    Q, _, mom, _ = gpu_solve(dvm, g, 0.7, 8)
    assert_parity(Q, mom, ref, qtol=1e-8, utol=1e-9)
    # smallest legal grid (skewed schedule): the direct solve is the reference
    import oracle.dense as dn
    m = np.zeros((4, 4), np.uint8)
    m[1, 1] = 1
    from paper_1704_03126_amd.geometry import Geometry
    g2 = Geometry(m, True, 4.0)
    ref2 = dn.solve(m, 2.0, 6, periodic_y=True, cells_per_H=4.0)
    Q2, _, mom2, _ = gpu_solve(dvm, g2, 2.0, 6)
    assert abs(Q2 - ref2.Q) < 1e-9 * abs(ref2.Q)
    assert np.max(np.abs(mom2["u1"] - ref2.u1)) < 1e-9
    # narrow periodic porous cell whose plain source iteration diverges at
    # delta = 0.01 when it lags only the periodic seams (the oracle's order
    # and the default one); the wrap-around order converges: the direct solve
    # decides
    from paper_1704_03126_amd.geometry import porous_discs as pd
    g3 = pd(8, 0.7, 5)
    ref3 = dn.solve(g3.mask, 0.01, 6, periodic_y=True, cells_per_H=8.0)
    Q3, _, mom3, info3 = gpu_solve(dvm, g3, 0.01, 6, tol=1e-12, schedule=dvm.DVM_SCHED_WRAP)
    assert info3.status == "converged"
    assert abs(Q3 - ref3.Q) < 1e-8 * abs(ref3.Q)


def test_delta_field_and_padding(dvm):
    """Per-cell delta (reciprocal per update) and a velocity count that does
    not fill the last group (12x12 -> 36 per quadrant, padded to 64)."""
    g = porous_discs(40, 0.6, 7)
    dl = delta_field(g.mask.shape, 1005)
    ref = oracle_solve(g, dl, 12)
    Q, ka, mom, _ = gpu_solve(dvm, g, dl, 12)
    assert_parity(Q, mom, ref, qtol=1e-8, utol=1e-9)
    assert np.isnan(ka)


@pytest.mark.parametrize("vel,waves", [(8, 4), (4, 4), (2, 8)])
def test_launch_shapes_agree(dvm, vel, waves):
    g = rough_channel(48, 20, 4, 24)
    base = gpu_solve(dvm, g, 1.0, 16, tol=1e-12)
    other = gpu_solve(dvm, g, 1.0, 16, tol=1e-12, vel=vel, waves=waves)
    assert abs(base[0] - other[0]) < 1e-11 * abs(base[0])
    assert np.max(np.abs(base[2]["u1"] - other[2]["u1"])) < 1e-11


def test_bitwise_determinism_and_graphs(dvm):
    g = porous_discs(48, 0.6, 3)
    a = gpu_solve(dvm, g, 0.5, 8, tol=1e-10)
    b = gpu_solve(dvm, g, 0.5, 8, tol=1e-10)
    c = gpu_solve(dvm, g, 0.5, 8, tol=1e-10, graphs=False)
    assert a[0] == b[0] == c[0]
    assert np.array_equal(a[2]["u1"], b[2]["u1"]) and np.array_equal(a[2]["u1"], c[2]["u1"])


def test_batched_equals_single(dvm):
    gs = [rough_channel(40, 20, 4, 20), porous_discs(36, 0.6, 11), plane_channel(24, 1),
          rough_channel(70, 30, 6, 35)]
    ds = [0.3, 2.0, 1.0, 5.0]
    # the same launch shape in both contexts: the autotuner picks shapes by
    # timing, and another shape sums the moments in another order
    s = dvm.Solver(8, len(gs), tol=1e-11, vel_per_lane=4, waves_per_block=8)
    for i, g in enumerate(gs):
        s.set_geometry(i, g.mask, g.periodic_y, g.cells_per_H)
    infos = s.solve(-1, ds)
    assert all(i.status == "converged" for i in infos)
    for i, g in enumerate(gs):
        Qb, _ = s.flow_rate(i)
        mb = s.moments(i)
        Qs, _, ms, _ = gpu_solve(dvm, g, ds[i], 8, vel=4, waves=8)
        assert Qb == Qs
        assert np.array_equal(mb["u1"], ms["u1"])
        ref = oracle_solve(g, ds[i], 8)
        assert_parity(Qb, mb, ref, qtol=1e-8, utol=1e-9)
    s.close()


def test_shear_stress(dvm):
    g = rough_channel(32, 24, 5, 16)
    ref = oracle_solve(g, 1.0, 8)
    _, _, mom, _ = gpu_solve(dvm, g, 1.0, 8, shear=True)
    assert np.max(np.abs(mom["p12"] - ref.p12)) < 1e-8


def test_max_iter_then_resume(dvm):
    g = rough_channel(32, 16, 3, 16)
    s = dvm.Solver(8, 1, tol=1e-11, max_iter=7, block_iters=4)
    s.set_geometry(0, g.mask, False, 16.0)
    info = s.solve(0, 5.0, raise_on_noconv=False)
    assert info.status == "max_iter" and info.iters == 7
    s2 = dvm.Solver(8, 1, tol=1e-11)
    s2.set_geometry(0, g.mask, False, 16.0)
    ref = s2.solve(0, 5.0)
    # resume (warm) in slices of 5 iterations: reaches the same fixed point
    s.close()
    s3 = dvm.Solver(8, 1, tol=1e-11, max_iter=5)
    s3.set_geometry(0, g.mask, False, 16.0)
    for _ in range(2000):
        info = s3.solve(0, 5.0, warm=True, raise_on_noconv=False)
        if info.status == "converged":
            break
    assert info.status == "converged"
    assert abs(s3.flow_rate(0)[0] - s2.flow_rate(0)[0]) < 1e-9
    s2.close()
    s3.close()


@pytest.mark.parametrize("graphs", [True, False])
def test_resume_is_bitwise(dvm, graphs):
    """A solve stopped at max_iter and resumed warm continues the same
    iteration: 40 iterations in slices of 8 give bitwise the moments of 40
    uninterrupted ones (plain iteration, so nothing but the state carries
    over; a tolerance no iterate reaches)."""
    g = rough_channel(32, 16, 3, 16)
    kw = dict(tol=1e-300, block_iters=4, accel=dvm.DVM_ACCEL_NONE, use_graphs=graphs,
              vel_per_lane=4, waves_per_block=8)
    a = dvm.Solver(8, 1, max_iter=40, **kw)
    a.set_geometry(0, g.mask, False, 16.0)
    ia = a.solve(0, 5.0, raise_on_noconv=False)
    assert ia.status == "max_iter" and ia.iters == 40
    b = dvm.Solver(8, 1, max_iter=8, **kw)
    b.set_geometry(0, g.mask, False, 16.0)
    ib = b.solve(0, 5.0, raise_on_noconv=False)
    for _ in range(4):
        ib = b.solve(0, 5.0, warm=True, raise_on_noconv=False)
    assert ib.status == "max_iter"
    ma, mb = a.moments(0), b.moments(0)
    for k in ("rho", "u1", "u2", "tau"):
        assert np.array_equal(ma[k], mb[k]), k
    assert a.flow_rate(0)[0] == b.flow_rate(0)[0]
    a.close()
    b.close()


def test_warm_start_delta_sweep(dvm):
    g = rough_channel(48, 24, 5, 24)
    s = dvm.Solver(8, 1, tol=1e-11)
    s.set_geometry(0, g.mask, False, 24.0)
    s.solve(0, 1.0)
    info = s.solve(0, 2.0, warm=True)
    Qw = s.flow_rate(0)[0]
    ref = oracle_solve(g, 2.0, 8)
    assert abs(Qw - ref.Q) < 1e-8 * abs(ref.Q)
    s.close()


@pytest.mark.parametrize("case", ["rough", "porous"])
def test_wrap_schedule_same_fixed_point(dvm, case):
    """The wrap-around diagonal lags different couplings but converges (on
    these geometries) to the same discrete solution as the oracle."""
    if case == "rough":
        g, nv = rough_channel(64, 32, 6, 32), 16
    else:
        g, nv = porous_discs(64, 0.6, 1003), 12
    ref = oracle_solve(g, 1.0, nv)
    Q, _, mom, info = gpu_solve(dvm, g, 1.0, nv, schedule=dvm.DVM_SCHED_WRAP)
    assert info.status == "converged"
    assert_parity(Q, mom, ref, qtol=1e-8, utol=1e-8)


def test_block_in_periodic_cell_default_schedule(dvm):
    """A solid block inside a periodic cell: the default schedule converges
    to the oracle's solution (the wrap-around diagonal diverges here)."""
    g = _block_cell()
    ref = oracle_solve(g, 0.7, 8)
    Q, _, mom, info = gpu_solve(dvm, g, 0.7, 8)
    assert info.status == "converged"
    assert_parity(Q, mom, ref, qtol=1e-8, utol=1e-8)


def _block_cell():
    from paper_1704_03126_amd.geometry import Geometry
    m = np.zeros((16, 16), np.uint8)
    m[6:10, 4:10] = 1
    return Geometry(mask=m, periodic_y=True, cells_per_H=16.0)


def test_auto_schedule_moves_runaway_instance_to_skew(dvm):
    """Default schedule without Krylov acceleration: the block-in-periodic
    cell runs away on the wrap-around diagonal, is moved to the skewed order
    and converges to the oracle's solution.  A second instance solved earlier
    keeps its solution through the new layout, and a well-behaved instance in
    a batch with it stays on the wrap-around diagonal and converges too."""
    gb, gr = _block_cell(), rough_channel(32, 16, 3, 16)
    refb = oracle_solve(gb, 0.7, 8)
    refr = oracle_solve(gr, 1.0, 8)
    s = dvm.Solver(8, 2, tol=1e-11, accel=dvm.DVM_ACCEL_NONE)
    s.set_geometry(0, gb.mask, gb.periodic_y, gb.cells_per_H)
    s.set_geometry(1, gr.mask, gr.periodic_y, gr.cells_per_H)
    info_r = s.solve(1, 1.0)
    Qr = s.flow_rate(1)[0]
    mr = s.moments(1)
    info_b = s.solve(0, 0.7)
    assert info_r.status == "converged" and info_b.status == "converged"
    assert info_r.schedule == "wrap" and info_b.schedule == "skew"
    assert_parity(s.flow_rate(0)[0], s.moments(0), refb, qtol=1e-8, utol=1e-8)
    # instance 1 untouched by the relayout: bit-identical moments
    assert s.flow_rate(1)[0] == Qr
    assert np.array_equal(s.moments(1)["u1"], mr["u1"])
    assert_parity(Qr, mr, refr, qtol=1e-8, utol=1e-8)
    # both at once, cold
    infos = s.solve(-1, [0.7, 1.0])
    assert all(i.status == "converged" for i in infos), infos
    assert [i.schedule for i in infos] == ["skew", "wrap"]
    assert_parity(s.flow_rate(0)[0], s.moments(0), refb, qtol=1e-8, utol=1e-8)
    assert_parity(s.flow_rate(1)[0], s.moments(1), refr, qtol=1e-8, utol=1e-8)
    s.close()


def test_autotuner_cache(dvm, tmp_path):
    """Default shape selection: the tuned solve equals an explicit-shape
    solve to round-off, writes its choice to the cache file, and a new
    context reads it back."""
    g = rough_channel(64, 32, 6, 32)
    cache = str(tmp_path / "tune.txt")
    s = dvm.Solver(12, 1, tol=1e-11, tune_cache=cache)
    s.set_geometry(0, g.mask, g.periodic_y, g.cells_per_H)
    s.solve(0, 1.0)
    Q1 = s.flow_rate(0)[0]
    s.close()
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and "|" in lines[0]
    V, G, V32, G32 = map(int, lines[0].split("|")[1].split())
    assert (V, G) in [(4, 8), (8, 4), (4, 4), (2, 8)] and V * G == V32 * G32
    Q2, _, _, _ = gpu_solve(dvm, g, 1.0, 12, vel=V, waves=G)
    assert abs(Q1 - Q2) <= 1e-12 * abs(Q2)
    s = dvm.Solver(12, 1, tol=1e-11, tune_cache=cache)
    s.set_geometry(0, g.mask, g.periodic_y, g.cells_per_H)
    s.solve(0, 1.0)
    s.close()
    assert len(open(cache).read().strip().splitlines()) == 1


def test_profile_counts_real_sweeps_and_launch_shape(dvm):
    """Profile mode times exactly the sweeps that did work (one per
    iteration), and the launch-shape query reports the tuned shape."""
    g = rough_channel(64, 32, 6, 32)
    s = dvm.Solver(12, 1, tol=1e-10, profile=True)
    s.set_geometry(0, g.mask, g.periodic_y, g.cells_per_H)
    assert s.launch_shape() == ((0, 0), (0, 0))        # autotuned, not chosen yet
    info = s.solve(0, 1.0)
    p = s.profile()
    (V, G), (V32, G32) = s.launch_shape()
    s.close()
    assert info.status == "converged"
    assert p["n_sweeps"] == info.iters and p["sweep_ms"] > 0 and p["other_ms"] > 0
    assert p["updates"] == info.iters * g.n_fluid * 12 * 12
    assert p["n_sweeps32"] == 0 and p["updates32"] == 0
    assert (V, G) in [(4, 8), (8, 4), (4, 4), (2, 8)] and V * G == V32 * G32
    # FP32 refinement: its FP32 correction sweeps and FP64 outer steps are
    # timed apart, and every sweep of the solve is counted once
    s = dvm.Solver(12, 1, tol=1e-10, profile=True, precision=dvm.DVM_FP32_REFINE)
    s.set_geometry(0, g.mask, g.periodic_y, g.cells_per_H)
    info = s.solve(0, 1.0)
    p = s.profile()
    s.close()
    assert info.status == "converged"
    assert p["n_sweeps"] == info.sweeps_fp64 and p["n_sweeps32"] == info.iters - info.sweeps_fp64
    assert p["updates32"] == p["n_sweeps32"] * g.n_fluid * 144 and p["sweep32_ms"] > 0


def test_largest_velocity_grid_and_narrow_channel(dvm):
    """The largest velocity grid (128 x 128 nodes, 16384 velocities) on a
    narrow rough channel of 5 columns (skewed order: fewer than 8 columns),
    with Maxwell walls, against the oracle."""
    g = rough_channel(5, 18, 3, 2)
    nv = 128
    ref = oracle.si_solve(g.mask, 0.8, nv, periodic_y=False, cells_per_H=g.cells_per_H,
                          alpha=0.9, tol=1e-12)
    Q, _, mom, info = gpu_solve(dvm, g, 0.8, nv, alpha=0.9)
    assert info.status == "converged" and info.schedule == "skew"
    assert_parity(Q, mom, ref, qtol=1e-9, utol=1e-9)


def test_dominant_mode_extrapolation(dvm):
    """Default acceleration at a delta where the source iteration settles on
    one slow mode: fewer sweeps than the plain iteration, the same fixed
    point (oracle), and no change where the rate never settles below 0.98."""
    g = rough_channel(64, 32, 6, 32)
    ref = oracle_solve(g, 10.0, 16)
    its = {}
    for acc in (dvm.DVM_ACCEL_NONE, dvm.DVM_ACCEL_AUTO):
        s = dvm.Solver(16, 1, tol=1e-11, accel=acc)
        s.set_geometry(0, g.mask, g.periodic_y, g.cells_per_H)
        info = s.solve(0, 10.0)
        Q = s.flow_rate(0)[0]
        mom = s.moments(0)
        s.close()
        assert info.status == "converged"
        assert_parity(Q, mom, ref, qtol=1e-9, utol=1e-9)
        its[acc] = info.iters
    assert its[dvm.DVM_ACCEL_AUTO] < 0.85 * its[dvm.DVM_ACCEL_NONE], its
