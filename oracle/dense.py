"""Explicit assembly of the discrete steady linearized-BGK problem (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).  This is a second,
independent coding of the discrete problem that the source iteration in
``dvm_oracle.c`` converges to: instead of sweeping, every coupling is written
as a matrix entry and the steady system is solved directly on tiny grids.

Unknowns are h[(f, k)] for fluid cell f (row-major order) and velocity
k = i * nv + j with (xi, eta) = (v_i, v_j).  For each unknown the row reads

    delta_c h_ck + (v . grad h)_ck - delta_c E_k(m_c) = g1 xi_k + g2 eta_k

(paper Eq. (BGK) without the time derivative, Eq. (iteration) at its fixed
point), with
  * E_k the discrete-conservative local equilibrium (paper Eq. (BGK) gain
    term divided by delta), a reading that reduces to
    rho + 2 u.v + tau (|v|^2 - 1) for exact quadrature;
  * the second-order upwind difference of Sec. II.A (text after
    Eq. (iteration)) in flux form, first-order face values next to walls on
    the staircase (reading);
  * diffuse walls of Eq. (diffuse2) with a Maxwell specular share 1 - alpha
    (reading for alpha < 1);
  * drive (g1, g2) = (1, 0): unit pressure gradient along x (reading; the
    paper defers the Poiseuille source to its ref. LeiComment2017 and fixes
    the normalisation through k_a and H* in Sec. III).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


def quad(nv: int):
    """Eq. (nonuniform_v) nodes, trapezoid-in-s weights, Maxwellian weights."""
    if nv < 4 or nv % 2:
        raise ValueError("nv must be even and >= 4")
    j = np.arange(nv)
    s = (2 * j - nv + 1) / (nv - 1)
    v = 4.0 * s ** 3
    w = 12.0 * s ** 2 * (2.0 / (nv - 1))
    w[0] *= 0.5
    w[-1] *= 0.5
    XI, ETA = np.meshgrid(v, v, indexing="ij")
    Wm = np.outer(w, w) * np.exp(-XI ** 2 - ETA ** 2) / np.pi
    xi, eta, W = XI.ravel(), ETA.ravel(), Wm.ravel()
    q = xi ** 2 + eta ** 2
    m0, m2, M2, M4 = W.sum(), (W * xi ** 2).sum(), (W * q).sum(), (W * q * q).sum()
    c2 = M2 / m0
    c4 = M4 - M2 * M2 / m0
    D = (W * xi * (xi > 0)).sum()
    return dict(v=v, w=w, xi=xi, eta=eta, W=W, q=q, m0=m0, m2=m2, M2=M2,
                M4=M4, c2=c2, c4=c4, D=D, nv=nv, K=nv * nv)


def equilibrium_matrix(Q):
    """P[k, k'] with E_k = sum_k' P[k, k'] h_k' (discrete-conservative gain)."""
    xi, eta, q, W = Q["xi"], Q["eta"], Q["q"], Q["W"]
    m0, m2, c2, c4 = Q["m0"], Q["m2"], Q["c2"], Q["c4"]
    # E = rho/m0 + (u1 xi + u2 eta)/m2 + t (q - c2),  t = (e - c2 rho)/c4
    basis_rho = 1.0 / m0 - c2 * (q - c2) / c4      # coefficient of rho in E_k
    basis_e = (q - c2) / c4                         # coefficient of e in E_k
    P = (np.outer(basis_rho, W) + np.outer(xi / m2, W * xi)
         + np.outer(eta / m2, W * eta) + np.outer(basis_e, W * q))
    return P


@dataclass
class System:
    A: sp.csr_matrix        # steady operator on [h; g] (cells then wall faces)
    dA_dalpha: sp.csr_matrix
    T: sp.csr_matrix        # transport rows only (h rows), incl. face coupling
    s: np.ndarray           # drive on cell rows; moving-wall source on face rows
    fluid: np.ndarray       # (nf, 2) cell coordinates (y, x)
    cell_index: np.ndarray  # (ny, nx) -> fluid index or -1
    faces: list             # [(f, side)] wall faces; side 0 W, 1 E, 2 S, 3 N
    delta_f: np.ndarray     # delta per fluid cell
    Q: dict
    nx: int
    ny: int
    dx: float
    P: np.ndarray
    nh: int                 # number of cell unknowns nf * K
    ds_dalpha: np.ndarray = None   # d s / d alpha (moving walls)
    area: np.ndarray = None        # dA / L per fluid cell (flow-rate weights)


_STEP = {0: (0, -1), 1: (0, 1), 2: (-1, 0), 3: (1, 0)}   # side -> (dy, dx)


def _solid(mask, periodic_y, y, x):
    ny, nx = mask.shape
    x %= nx
    if y < 0 or y >= ny:
        if not periodic_y:
            return True
        y %= ny
    return bool(mask[y, x])


def assemble(mask, delta, nv, *, periodic_y=False, cells_per_H=None,
             alpha=1.0, drive=(1.0, 0.0), wall_velocity=(0.0, 0.0), dy=None) -> System:
    """Assemble the steady problem with explicit wall-face unknowns.

    Unknowns: h[f*K + k] for every fluid cell f and velocity k, then
    g[nh + phi*K + k], the value of h on wall face phi for a velocity k leaving
    that face (rows for velocities entering the face are g = 0 and unused).

    Transport (reading of the second-order upwind difference on the staircase,
    flux form): along each axis the velocity component a carries the face
    values |a| (h_out - h_in)/dx, where each face value is the linear
    extrapolation 1.5 h_u - 0.5 h_uu from the upwind cell u through its own
    upwind neighbour uu, or h_u when uu is solid; a wall face on the upwind
    side supplies g itself.  In the interior this is the paper's
    (3 h_c - 4 h_1 + h_2)/(2 dx).

    Walls (Eq. (diffuse2) and Maxwell's specular share as a reading):
    g = alpha * rho_w + (1 - alpha) * h_inc(mirror k), with
    rho_w = sum_inc W |v_n| h_inc / D and h_inc the reconstructed incident
    face value.  The outer bottom and top walls of a channel may slide
    along x at wall_velocity = (U_bottom, U_top); their diffuse part is then
    that of Eq. (diffuse1), rho_w + 2 U xi, a source term of the face rows.

    dy (optional): row heights in units of H.  Along y the face value
    extrapolated from the upwind cell u through uu is h_u + r (h_u - h_uu),
    r = dy_u / (dy_u + dy_uu) (1/2 on a uniform grid), and the flux
    difference is divided by the cell's own height.

    drive = (a, b) is the source a xi + b eta of every cell (pressure
    gradients along x and y; (1, 0) is the Poiseuille problem of Sec. III,
    (0, 0) with U_top = 1 the Couette problem of Sec. II).
    """
    mask = np.asarray(mask, dtype=np.uint8)
    ny, nx = mask.shape
    if cells_per_H is None:
        cells_per_H = float(ny)
    dx = 1.0 / cells_per_H
    hrow = np.full(ny, dx) if dy is None else np.asarray(dy, dtype=np.float64)
    Q = quad(nv)
    K = Q["K"]
    xi, eta, W, D = Q["xi"], Q["eta"], Q["W"], Q["D"]
    cell_index = -np.ones((ny, nx), dtype=np.int64)
    fluid = np.argwhere(mask == 0)
    for f, (y, x) in enumerate(fluid):
        cell_index[y, x] = f
    nf = len(fluid)
    nh = nf * K
    dfield = np.broadcast_to(np.asarray(delta, dtype=np.float64), (ny, nx))
    delta_f = np.array([dfield[y, x] for y, x in fluid])

    def nb(f, side, dist=1):
        y, x = fluid[f]
        dy, dxx = _STEP[side]
        yy, xx = y + dist * dy, x + dist * dxx
        if _solid(mask, periodic_y, yy, xx):
            return -1
        return int(cell_index[yy % ny, xx % nx])

    def axis_active(side):
        return not (side < 2 and nx == 1)

    faces = []
    face_id = {}
    for f in range(nf):
        for side in range(4):
            if axis_active(side) and nb(f, side) < 0:
                face_id[(f, side)] = len(faces)
                faces.append((f, side))
    N = nh + len(faces) * K

    def hid(f, k):
        return f * K + k

    def gid(f, side, k):
        return nh + face_id[(f, side)] * K + k

    def vcomp(side, k):
        return xi[k] if side < 2 else eta[k]

    def upwind_side(axis, k):
        v = xi[k] if axis == 0 else eta[k]
        return (0 if v > 0 else 1) if axis == 0 else (2 if v > 0 else 3)

    def leaves(side, k):
        # moving away from `side` (into the fluid from a wall on that side)
        v = vcomp(side, k)
        return v > 0 if side in (0, 2) else v < 0

    rows, cols, vals = [], [], []
    drows, dcols, dvals = [], [], []
    trows, tcols, tvals = [], [], []

    def add(r, c, v, t=False):
        rows.append(r); cols.append(c); vals.append(v)
        if t:
            trows.append(r); tcols.append(c); tvals.append(v)

    P = equilibrium_matrix(Q)
    IP = np.eye(K) - P
    for f in range(nf):
        for k in range(K):
            u = hid(f, k)
            if delta_f[f] != 0.0:
                for kk in range(K):
                    if IP[k, kk] != 0.0:
                        add(u, hid(f, kk), delta_f[f] * IP[k, kk])
            for axis in (0, 1):
                if axis == 0 and nx == 1:
                    continue
                side = upwind_side(axis, k)
                yc = fluid[f][0]
                if axis == 0:
                    c, rc, ru = abs(xi[k]) / dx, 0.5, 0.5
                else:
                    step = _STEP[side][0]
                    y1, y2 = (yc + step) % ny, (yc + 2 * step) % ny
                    c = abs(eta[k]) / hrow[yc]
                    rc = hrow[yc] / (hrow[yc] + hrow[y1])
                    ru = hrow[y1] / (hrow[y1] + hrow[y2])
                f1 = nb(f, side, 1)
                if f1 < 0:                      # wall face on the upwind side
                    add(u, u, 1.0 * c, True)
                    add(u, gid(f, side, k), -1.0 * c, True)
                    continue
                f2 = nb(f, side, 2)
                if f2 < 0:                      # upwind neighbour touches a wall
                    add(u, u, (1.0 + rc) * c, True)
                    add(u, hid(f1, k), -(1.0 + rc) * c, True)
                else:
                    add(u, u, (1.0 + rc) * c, True)
                    add(u, hid(f1, k), -(1.0 + rc + ru) * c, True)
                    add(u, hid(f2, k), ru * c, True)

    nv_ = nv
    for phi, (f, side) in enumerate(faces):
        opp = side ^ 1
        fo = nb(f, opp, 1)
        inc = [k for k in range(K) if not leaves(side, k)]

        # incident face value extrapolated across the wall cell (through its
        # neighbour opposite the face)
        if side >= 2 and fo >= 0:
            rface = hrow[fluid[f][0]] / (hrow[fluid[f][0]] + hrow[fluid[fo][0]])
        else:
            rface = 0.5

        def h_inc_terms(k):
            # incident face value as a combination of unknowns
            if fo < 0:
                return [(hid(f, k), 1.0)]
            return [(hid(f, k), 1.0 + rface), (hid(fo, k), -rface)]

        for k in range(K):
            r = gid(f, side, k)
            add(r, r, 1.0)
            if not leaves(side, k):
                continue
            i, j = divmod(k, nv_)
            km = ((nv_ - 1 - i) * nv_ + j) if side < 2 else (i * nv_ + (nv_ - 1 - j))
            for kk in inc:
                a_d = W[kk] * abs(vcomp(side, kk)) / D      # diffuse weight
                a_s = 1.0 if kk == km else 0.0             # specular weight
                wv = alpha * a_d + (1.0 - alpha) * a_s
                dv = a_d - a_s
                for col, cf in h_inc_terms(kk):
                    if wv != 0.0:
                        add(r, col, -wv * cf)
                    if dv != 0.0:
                        drows.append(r); dcols.append(col); dvals.append(-dv * cf)

    A = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    dA = sp.csr_matrix((dvals, (drows, dcols)), shape=(N, N))
    T = sp.csr_matrix((tvals, (trows, tcols)), shape=(N, N))
    s = np.zeros(N)
    s[:nh] = np.tile(drive[0] * xi + drive[1] * eta, nf)
    ds = np.zeros(N)                    # d s / d alpha
    if not periodic_y:
        for phi, (f, side) in enumerate(faces):
            y = fluid[f][0]
            U = wall_velocity[0] if (side == 2 and y == 0) else \
                wall_velocity[1] if (side == 3 and y == ny - 1) else 0.0
            if U == 0.0:
                continue
            for k in range(K):
                if leaves(side, k):
                    ds[gid(f, side, k)] = 2.0 * U * xi[k]
    s += alpha * ds
    return System(A=A, dA_dalpha=dA, T=T, s=s, fluid=fluid, cell_index=cell_index,
                  faces=faces, delta_f=delta_f, Q=Q, nx=nx, ny=ny, dx=dx, P=P, nh=nh,
                  ds_dalpha=ds, area=hrow[fluid[:, 0]] / nx)


def _bordered_solve(M, rhs, g):
    N = M.shape[0]
    B = np.zeros((N + 1, N + 1))
    B[:N, :N] = M.toarray() if sp.issparse(M) else M
    B[:N, N] = g
    B[N, :N] = g
    r = np.concatenate([rhs, [0.0]])
    sol = np.linalg.solve(B, r)
    return sol[:N], sol[N]


@dataclass
class DenseResult:
    h: np.ndarray           # (nf, K)
    Q: float
    rho: np.ndarray         # (ny, nx) zero fluid mean
    u1: np.ndarray
    u2: np.ndarray
    border: float
    sys: System
    x: np.ndarray           # full solution [h; g]


def moments(sys: System, h):
    """Moments of Sec. II.A at every fluid cell: rho, u1, u2, e."""
    Q = sys.Q
    W, xi, eta, q = Q["W"], Q["xi"], Q["eta"], Q["q"]
    return (h @ W, h @ (W * xi), h @ (W * eta), h @ (W * q))


def solve(mask, delta, nv, **kw) -> DenseResult:
    sys = assemble(mask, delta, nv, **kw)
    K = sys.Q["K"]
    nf = len(sys.fluid)
    g = np.zeros(sys.A.shape[0])
    g[:sys.nh] = np.tile(sys.Q["W"], nf)   # gauge: sum of rho over fluid cells = 0
    xv, lam = _bordered_solve(sys.A, sys.s, g)
    h = xv[:sys.nh].reshape(nf, K)
    r, m1, m2, _ = moments(sys, h)
    rho = np.zeros((sys.ny, sys.nx)); u1 = np.zeros_like(rho); u2 = np.zeros_like(rho)
    for f, (y, x) in enumerate(sys.fluid):
        rho[y, x], u1[y, x], u2[y, x] = r[f], m1[f], m2[f]
    Qv = float(sys.area @ m1)            # (1/L) sum u1 dA, dA / L = dy / nx
    return DenseResult(h=h, Q=Qv, rho=rho, u1=u1, u2=u2, border=lam, sys=sys, x=xv)


@dataclass
class AdjointResult:
    lam: np.ndarray         # (nf, K) adjoint of A^T lam = dQ/dh
    dQ_ddelta: np.ndarray   # (ny, nx), zero in solids
    dQ_dalpha: float
    Q: float


def adjoint(mask, delta, nv, **kw) -> AdjointResult:
    """Discrete adjoint of the flow rate: A^T lam = dQ/dh, then
    dQ/dtheta = -lam^T (dA/dtheta h - ds/dtheta) for theta = delta_c and
    alpha (the source depends on alpha only through a moving wall)."""
    fwd = solve(mask, delta, nv, **kw)
    sys = fwd.sys
    K = sys.Q["K"]
    nf = len(sys.fluid)
    W, xi = sys.Q["W"], sys.Q["xi"]
    N = sys.A.shape[0]
    c = np.zeros(N)
    c[:sys.nh] = (sys.area[:, None] * (W * xi)[None, :]).ravel()
    g = np.zeros(N)
    g[:sys.nh] = np.tile(W, nf)
    lv, _ = _bordered_solve(sys.A.T, c, g)
    lam = lv[:sys.nh].reshape(nf, K)
    h = fwd.h
    E = h @ sys.P.T                    # E_k(m_c) for every fluid cell
    dd = -(lam * (h - E)).sum(axis=1)
    dQ_ddelta = np.zeros((sys.ny, sys.nx))
    for f, (y, x) in enumerate(sys.fluid):
        dQ_ddelta[y, x] = dd[f]
    dQ_dalpha = float(-lv @ (sys.dA_dalpha @ fwd.x - sys.ds_dalpha))
    return AdjointResult(lam=lam, dQ_ddelta=dQ_ddelta, dQ_dalpha=dQ_dalpha, Q=fwd.Q)
