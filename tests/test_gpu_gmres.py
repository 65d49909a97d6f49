"""GMRES-accelerated iteration on the GPU, through the C ABI.

Same sweeps, same discrete fixed point: the results are compared with the
FP64 oracle (its source iteration, or its direct solve where the lagged
iteration itself diverges) and with the plain iteration on the GPU.
"""
import numpy as np
import pytest

import oracle
import oracle.dense as dn
from paper_1704_03126_amd.geometry import (Geometry, delta_field, plane_channel,
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


def solve(dvm, g, delta, nv, alpha=1.0, tol=1e-10, **kw):
    s = dvm.Solver(nv, 1, tol=tol, accel=dvm.DVM_ACCEL_GMRES, **kw)
    s.set_geometry(0, g.mask, g.periodic_y, g.cells_per_H)
    info = s.solve(0, delta, alpha)
    Q, _ = s.flow_rate(0)
    mom = s.moments(0)
    return s, info, Q, mom


@pytest.mark.parametrize("case,delta,alpha", [
    ("rough", 0.1, 1.0), ("rough", 10.0, 1.0), ("rough", 1.0, 0.8),
    ("porous", 1.0, 1.0), ("plane", 1.0, 1.0)])
def test_gmres_matches_oracle(dvm, case, delta, alpha):
    if case == "rough":
        g, nv = rough_channel(64, 32, 6, 32), 12
    elif case == "porous":
        g, nv = porous_discs(64, 0.6, 1003), 8
    else:
        g, nv = plane_channel(64), 16
    ref = oracle.si_solve(g.mask, delta, nv, periodic_y=g.periodic_y,
                          cells_per_H=g.cells_per_H, alpha=alpha, tol=1e-12)
    s, info, Q, mom = solve(dvm, g, delta, nv, alpha)
    s.close()
    assert info.status == "converged", info
    assert abs(Q - ref.Q) <= 1e-8 * abs(ref.Q), (Q, ref.Q)
    assert np.max(np.abs(mom["u1"] - ref.u1)) <= 1e-8


def test_gmres_where_the_lagged_iteration_diverges(dvm):
    """Both sweep orders have a geometry on which the plain iteration
    diverges; GMRES on the same sweeps converges to the direct solution."""
    m = np.zeros((16, 16), np.uint8)
    m[6:10, 4:10] = 1
    g = Geometry(mask=m, periodic_y=True, cells_per_H=16.0)
    ref = oracle.si_solve(m, 0.7, 8, periodic_y=True, cells_per_H=16.0, tol=1e-12)
    s, info, Q, mom = solve(dvm, g, 0.7, 8, schedule=dvm.DVM_SCHED_WRAP)
    s.close()
    assert info.status == "converged"
    assert abs(Q - ref.Q) <= 1e-8 * abs(ref.Q)
    g3 = porous_discs(8, 0.7, 5)
    ref3 = dn.solve(g3.mask, 0.01, 6, periodic_y=True, cells_per_H=8.0)
    s, info, Q3, mom3 = solve(dvm, g3, 0.01, 6, tol=1e-12)
    s.close()
    assert info.status == "converged"
    assert abs(Q3 - ref3.Q) <= 1e-8 * abs(ref3.Q), (Q3, ref3.Q)
    assert np.max(np.abs(mom3["u1"] - ref3.u1)) <= 1e-8


def test_gmres_adjoint_multi_strip(dvm):
    """Adjoint of a three-strip periodic porous cell in the default order
    (the plain adjoint iteration diverges there): sum of dQ/d delta_c equals
    the derivative of the uniform problem."""
    g = porous_discs(130, 0.65, 1005)
    nv = 8
    s = dvm.Solver(nv, 1, tol=1e-12, accel=dvm.DVM_ACCEL_GMRES)
    s.set_geometry(0, g.mask, g.periodic_y, g.cells_per_H)
    s.solve(0, 1.0, 0.9)
    gd, ga = s.grad(0)
    eps = 1e-4
    s.solve(0, 1.0 + eps, 0.9)
    qp = s.flow_rate(0)[0]
    s.solve(0, 1.0 - eps, 0.9)
    qm = s.flow_rate(0)[0]
    # dQ/d alpha is small (about 1e-5 of Q): a fourth-order central
    # difference at step 1e-2 keeps both its truncation error and the solves'
    # own error (tol 1e-12 on u1) well below 1e-6 of the derivative, which a
    # second-order one at step 1e-4 could not (its solve-error term alone
    # is about 1e-3 of it unless the errors of neighbouring solves cancel)
    ea = 1e-2
    qa = {}
    for k in (-2, -1, 1, 2):
        s.solve(0, 1.0, 0.9 + k * ea)
        qa[k] = s.flow_rate(0)[0]
    s.close()
    fd = (qp - qm) / (2 * eps)
    assert abs(gd.sum() - fd) <= 1e-6 * abs(fd), (gd.sum(), fd)
    fda = (8.0 * (qa[1] - qa[-1]) - (qa[2] - qa[-2])) / (12.0 * ea)
    assert abs(ga - fda) <= 1e-6 * abs(fda), (ga, fda)


def test_gmres_batched_equals_single(dvm):
    """A batch solved by GMRES matches the oracle, and every instance's
    result is bitwise that of its own single-instance solve: each instance
    runs its own Arnoldi process (own restart columns, own stop, own kept
    harmonic Ritz vectors); the batch only shares the sweeps.  The last
    instance (delta 40) restarts many times with deflation."""
    gs = [rough_channel(48, 24, 4, 24), porous_discs(40, 0.6, 1010), plane_channel(16),
          porous_discs(48, 0.6, 1003)]
    deltas = [0.5, 2.0, 1.0, 40.0]
    nv = 8
    shape = dict(vel_per_lane=4, waves_per_block=8)   # the same sweep layout in both contexts
    b = dvm.Solver(nv, len(gs), tol=1e-10, accel=dvm.DVM_ACCEL_GMRES, **shape)
    for i, g in enumerate(gs):
        b.set_geometry(i, g.mask, g.periodic_y, g.cells_per_H)
    infos = b.solve(-1, deltas)
    Qb = [b.flow_rate(i)[0] for i in range(len(gs))]
    ub = [b.moments(i)["u1"] for i in range(len(gs))]
    b.close()
    for i, g in enumerate(gs):
        assert infos[i].status == "converged"
        ref = oracle.si_solve(g.mask, deltas[i], nv, periodic_y=g.periodic_y,
                              cells_per_H=g.cells_per_H, tol=1e-12)
        assert abs(Qb[i] - ref.Q) <= 1e-8 * abs(ref.Q), (i, Qb[i], ref.Q)
        s, info, Q1, mom1 = solve(dvm, g, deltas[i], nv, **shape)
        s.close()
        assert Q1 == Qb[i], (i, Q1, Qb[i])
        assert np.array_equal(mom1["u1"], ub[i]), i


def test_auto_hands_diverging_instances_to_gmres(dvm):
    """Default mode: the plain iteration runs, stops contracting on the two
    geometries above, and GMRES finishes them; a well-behaved instance in the
    same batch stays on the plain iteration."""
    m = np.zeros((16, 16), np.uint8)
    m[6:10, 4:10] = 1
    gs = [Geometry(mask=m, periodic_y=True, cells_per_H=16.0), rough_channel(32, 16, 3, 16)]
    s = dvm.Solver(8, 2, tol=1e-10, schedule=dvm.DVM_SCHED_WRAP)
    for i, g in enumerate(gs):
        s.set_geometry(i, g.mask, g.periodic_y, g.cells_per_H)
    infos = s.solve(-1, [0.7, 1.0])
    Qs = [s.flow_rate(i)[0] for i in range(2)]
    s.close()
    for i, g in enumerate(gs):
        assert infos[i].status == "converged", infos[i]
        ref = oracle.si_solve(g.mask, [0.7, 1.0][i], 8, periodic_y=g.periodic_y,
                              cells_per_H=g.cells_per_H, tol=1e-12)
        assert abs(Qs[i] - ref.Q) <= 1e-8 * abs(ref.Q), (i, Qs[i], ref.Q)
    g3 = porous_discs(8, 0.7, 5)
    ref3 = dn.solve(g3.mask, 0.01, 6, periodic_y=True, cells_per_H=8.0)
    s = dvm.Solver(6, 1, tol=1e-12)
    s.set_geometry(0, g3.mask, True, 8.0)
    info = s.solve(0, 0.01)
    Q3 = s.flow_rate(0)[0]
    s.close()
    assert info.status == "converged"
    assert abs(Q3 - ref3.Q) <= 1e-8 * abs(ref3.Q)


def test_auto_gmres_trial_on_slow_iteration(dvm):
    """A periodic porous cell (199^2, seeded, 48^2 velocities) at delta 3.69
    whose plain iteration contracts at about 0.9986 per sweep (some 11000
    sweeps to tol 1e-8): AUTO hands it to GMRES on trial, GMRES keeps it
    (its cycles reduce the residual faster per second than the plain rate),
    and the result is GMRES's own to within the tolerance.  Also a solve of
    the batch that holds it next to a fast instance: the fast one converges
    plain and the counts stay per instance."""
    from paper_1704_03126_amd.geometry import batch_instances
    g = batch_instances(64)[6]
    assert (g.ny, g.nx) == (199, 199) and g.periodic_y
    d = g.meta["delta"]
    res = {}
    for name, acc in (("auto", dvm.DVM_ACCEL_AUTO), ("gmres", dvm.DVM_ACCEL_GMRES)):
        s = dvm.Solver(48, 1, tol=1e-8, max_iter=30000, accel=acc)
        s.set_geometry(0, g.mask, g.periodic_y, g.cells_per_H)
        info = s.solve(0, d)
        assert info.status == "converged", (name, info)
        res[name] = (s.flow_rate(0)[0], info.iters)
        s.close()
    (qa, ia), (qg, ig) = res["auto"], res["gmres"]
    assert abs(qa - qg) <= 1e-8 * abs(qg), (qa, qg)
    assert ia < 2000, ia
    g1 = rough_channel(64, 32, 6, 32)
    s = dvm.Solver(48, 2, tol=1e-8, max_iter=30000)
    s.set_geometry(0, g.mask, g.periodic_y, g.cells_per_H)
    s.set_geometry(1, g1.mask, g1.periodic_y, g1.cells_per_H)
    infos = s.solve(-1, [d, 1.0])
    q0, q1 = s.flow_rate(0)[0], s.flow_rate(1)[0]
    s.close()
    assert all(i.status == "converged" for i in infos), infos
    assert abs(q0 - qg) <= 1e-8 * abs(qg), (q0, qg)
    assert 0 < infos[1].iters < 200 and infos[0].iters < 2000, infos
    s = dvm.Solver(48, 1, tol=1e-8)
    s.set_geometry(0, g1.mask, g1.periodic_y, g1.cells_per_H)
    s.solve(0, 1.0)
    assert abs(s.flow_rate(0)[0] - q1) <= 1e-9 * abs(q1)
    s.close()


def test_gmres_deflated_restarts(dvm):
    """Deflated restarts (harmonic Ritz vectors kept from cycle to cycle)
    against plain restarts on a periodic porous cell at large delta, where
    restarted GMRES(64) stagnates: both reach the oracle's fixed point, the
    deflated one in fewer sweeps."""
    g = porous_discs(48, 0.6, 1003)
    nv = 8
    ref = oracle.si_solve(g.mask, 40.0, nv, periodic_y=True, cells_per_H=48.0, tol=1e-12)
    res = {}
    for name, kd in (("plain", -1), ("deflated", 0), ("deflated8", 8)):
        s, info, Q, mom = solve(dvm, g, 40.0, nv, krylov_deflate=kd)
        s.close()
        assert info.status == "converged", (name, info)
        assert abs(Q - ref.Q) <= 1e-8 * abs(ref.Q), (name, Q, ref.Q)
        assert np.max(np.abs(mom["u1"] - ref.u1)) <= 1e-8, name
        res[name] = info.iters
    assert res["deflated"] < res["plain"], res
    assert res["deflated8"] < res["plain"], res
    # deeper in the slow regime (no oracle run: the plain iteration would
    # need tens of thousands of sweeps): the same fixed point, far fewer sweeps
    out = {}
    for name, kd in (("plain", -1), ("deflated", 0)):
        s, info, Q, mom = solve(dvm, g, 150.0, nv, krylov_deflate=kd)
        s.close()
        assert info.status == "converged", (name, info)
        out[name] = (Q, info.iters, mom["u1"])
    (qp, ip, up), (qd, idf, ud) = out["plain"], out["deflated"]
    assert abs(qd - qp) <= 1e-8 * abs(qp), (qd, qp)
    assert np.max(np.abs(ud - up)) <= 1e-8
    assert idf < 0.8 * ip, (idf, ip)


@pytest.mark.parametrize("m,kd", [(8, 1), (12, 0), (16, 7), (64, 31), (40, -1)])
def test_gmres_restart_shapes(dvm, m, kd):
    """Restart lengths and kept counts at the edges of their ranges (one
    kept vector, a kept count one short of half the restart, the largest
    kept count) reach the oracle's fixed point on the large-delta porous
    cell; kd = 0 keeps a quarter of the restart, kd < 0 restarts plainly.
    (Much shorter restarts do not stop here: the stop rule divides the
    change by the smallest singular value of the cycle's projection, which
    a four-step cycle underestimates.)"""
    g = porous_discs(48, 0.6, 1003)
    nv = 8
    ref = _ref48(g)
    s, info, Q, mom = solve(dvm, g, 40.0, nv, krylov_dim=m, krylov_deflate=kd, max_iter=40000)
    s.close()
    assert info.status == "converged", info
    assert abs(Q - ref.Q) <= 1e-8 * abs(ref.Q), (Q, ref.Q)
    assert np.max(np.abs(mom["u1"] - ref.u1)) <= 1e-8


_REF48 = {}


def _ref48(g):
    if "r" not in _REF48:
        _REF48["r"] = oracle.si_solve(g.mask, 40.0, 8, periodic_y=True, cells_per_H=48.0, tol=1e-12)
    return _REF48["r"]
