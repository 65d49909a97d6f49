"""Pins of the oracle's Couette problem (Sec. II): a channel whose outer top
wall slides along x at U (Eq. diffuse1, U0/v_m = 1) and no pressure gradient.

* Smooth channel: the problem splits into the uniform drift h0 = (U_b + U_t) xi
  (the exact discrete solution when both walls slide at (U_b + U_t)/2: the
  discrete-conservative equilibrium reproduces it) plus a problem with walls at
  -/+ (U_t - U_b)/2 whose u1 profile is odd about the centreline.  Hence
  Q_s = (U_b + U_t) m2 at every delta (the paper's "Q_s = 0.5" for U_t = 1,
  where exact quadrature has m2 = 1/2) and u1(y) + u1(mirror y) =
  2 (U_b + U_t) m2 row by row.
* Free-molecular limit: every molecule going up carries the bottom wall's
  drift and every molecule going down the top's, so u1 is uniform.
* Linearity: Couette + Poiseuille = the problem with both sources.
* The source iteration equals the direct solve with the moving wall as a
  source on the wall-face rows, and the dense adjoint's d Q / d alpha (which
  now includes d s / d alpha) equals finite differences.
"""
import numpy as np
import pytest

import oracle
import oracle.dense as dn
from paper_1704_03126_amd.geometry import (fractal_couette_channel, plane_channel,
                                           rough_channel)


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


COUETTE = dict(drive=0.0, wall_velocity=(0.0, 1.0))


@pytest.mark.parametrize("delta", [0.0, 0.1, 1.0, 10.0])
def test_smooth_couette_flow_rate_is_m2(delta):
    nv = 16
    g = plane_channel(24)
    m2 = oracle.quadrature(nv).m2
    r = oracle.si_solve(g.mask, delta, nv, tol=1e-14, max_iter=100000, **COUETTE)
    assert r.converged
    assert abs(r.Q - m2) <= 2e-13, (r.Q, m2)
    # odd part about the centreline: u1(y) + u1(ny-1-y) = 2 m2
    u = r.u1[:, 0]
    assert np.max(np.abs(u + u[::-1] - 2 * m2)) <= 1e-12
    # the fluid is dragged by the top wall: u1 grows towards it
    if delta > 0:
        assert np.all(np.diff(u) > 0)


def test_free_molecular_uniform_drift():
    nv = 12
    m2 = oracle.quadrature(nv).m2
    r = oracle.si_solve(plane_channel(16).mask, 0.0, nv, tol=1e-14,
                        drive=0.0, wall_velocity=(0.3, 0.9))
    assert np.max(np.abs(r.u1[:, 0] - 1.2 * m2)) <= 1e-13


def test_general_wall_speeds_and_sign():
    nv = 12
    m2 = oracle.quadrature(nv).m2
    r = oracle.si_solve(plane_channel(16).mask, 2.0, nv, tol=1e-14,
                        drive=0.0, wall_velocity=(-0.4, 1.0))
    assert abs(r.Q - 0.6 * m2) <= 1e-13
    assert r.u1[0, 0] < 0 < r.u1[-1, 0]


def test_superposition_with_poiseuille():
    g = rough_channel(16, 12, 2, 8)
    kw = dict(periodic_y=False, cells_per_H=g.cells_per_H, alpha=0.8, tol=1e-14)
    both = oracle.si_solve(g.mask, 1.0, 8, drive=1.0, wall_velocity=(0.0, 1.0), **kw)
    pois = oracle.si_solve(g.mask, 1.0, 8, **kw)
    cou = oracle.si_solve(g.mask, 1.0, 8, **COUETTE, **kw)
    assert np.max(np.abs(both.u1 - pois.u1 - cou.u1)) <= 1e-12
    assert abs(both.Q - pois.Q - cou.Q) <= 1e-12


@pytest.mark.parametrize("alpha", [1.0, 0.8])
def test_source_iteration_equals_direct_solve(alpha):
    m = rough_channel(8, 8, 2, 4).mask
    d = dn.solve(m, 0.7, 6, alpha=alpha, drive=(0.0, 0.0), wall_velocity=(0.0, 1.0))
    s = oracle.si_solve(m, 0.7, 6, alpha=alpha, tol=1e-14, **COUETTE)
    assert abs(d.Q - s.Q) <= 1e-13
    assert np.max(np.abs(d.u1 - s.u1)) <= 1e-13
    assert np.max(np.abs(d.u2 - s.u2)) <= 1e-13


def test_dense_adjoint_alpha_derivative_with_sliding_wall():
    m = rough_channel(8, 8, 2, 4).mask
    kw = dict(drive=(0.0, 0.0), wall_velocity=(0.0, 1.0))
    a = dn.adjoint(m, 0.7, 6, alpha=0.8, **kw)
    e = 1e-6
    qp = dn.solve(m, 0.7, 6, alpha=0.8 + e, **kw).Q
    qm = dn.solve(m, 0.7, 6, alpha=0.8 - e, **kw).Q
    assert abs(a.dQ_dalpha - (qp - qm) / (2 * e)) <= 1e-7 * abs(a.dQ_dalpha)
    # d Q / d delta of one cell against finite differences
    base = np.full(m.shape, 0.7)
    y, x = 4, 5
    dp, dm_ = base.copy(), base.copy()
    dp[y, x] += e
    dm_[y, x] -= e
    fd = (dn.solve(m, dp, 6, alpha=0.8, **kw).Q - dn.solve(m, dm_, 6, alpha=0.8, **kw).Q) / (2 * e)
    assert abs(a.dQ_ddelta[y, x] - fd) <= 1e-6 * abs(fd) + 1e-12


def test_rough_wall_slows_the_flow():
    """Fractal staircase on the resting wall: Q_r < Q_s, and the flow rate
    rises towards Q_s as the roughness shrinks."""
    nv = 8
    m2 = oracle.quadrature(nv).m2
    qs = []
    for eps in (0.06, 0.02):
        g = fractal_couette_channel(16, eps=eps)
        r = oracle.si_solve(g.mask, 1.0, nv, cells_per_H=g.cells_per_H, tol=1e-12, **COUETTE)
        qs.append(r.Q)
    assert qs[0] < qs[1] < m2
