"""CPU oracle for the linearized-BGK discrete velocity method (FP64).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package.  It shares no code
with the GPU solver (``paper_1704_03126_amd``) and the GPU solver never
imports it.

Two independent codings of the same discrete problem live here:
  * ``dvm_oracle.c`` (loaded through ctypes): the paper's source iteration,
    Eq. (iteration), with per-velocity upwind sweeps -- the plain, slow
    reference the GPU is compared against;
  * ``dense.py``: explicit sparse/dense assembly of the steady operator and a
    direct solve on tiny grids, used to pin the iteration, and the discrete
    adjoint for gradient checks.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dvm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
               "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.oracle_quadrature.argtypes = [ctypes.c_int, P, P, P, P, P, P]
        lib.oracle_codes.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P]
        D = ctypes.c_double
        lib.oracle_si_solve.argtypes = [
            ctypes.c_int, ctypes.c_int, P, ctypes.c_int, D, P,
            ctypes.c_int, P, ctypes.c_int, D, D, D, D, D,
            ctypes.c_long, P, P, P, P, P, P, P, P]
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Quadrature:
    nv: int
    v: np.ndarray
    w1: np.ndarray
    xi: np.ndarray
    eta: np.ndarray
    W: np.ndarray
    m0: float
    m2: float
    M2: float
    M4: float
    c2: float
    c4: float
    D: float


def quadrature(nv: int) -> Quadrature:
    """Velocity grid of Eq. (nonuniform_v) with trapezoid-in-s weights."""
    lib = _load()
    K = nv * nv
    v = np.zeros(nv)
    w1 = np.zeros(nv)
    xi = np.zeros(K)
    eta = np.zeros(K)
    W = np.zeros(K)
    cs = np.zeros(7)
    if lib.oracle_quadrature(nv, _ptr(v), _ptr(w1), _ptr(xi), _ptr(eta), _ptr(W), _ptr(cs)):
        raise ValueError("nv must be even and >= 4")
    return Quadrature(nv, v, w1, xi, eta, W, *cs)


def codes(mask: np.ndarray, periodic_y: bool) -> np.ndarray:
    """Per-cell stencil codes (W, E, S, N): 0 2nd-order, 1 1st-order, 2 wall, 3 none."""
    lib = _load()
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    ny, nx = m.shape
    out = np.zeros((ny, nx, 4), dtype=np.uint8)
    if lib.oracle_codes(nx, ny, _ptr(m), int(periodic_y), _ptr(out)):
        raise ValueError("bad geometry")
    return out


@dataclass
class SIResult:
    Q: float
    rho: np.ndarray
    u1: np.ndarray
    u2: np.ndarray
    tau: np.ndarray
    p12: np.ndarray
    iters: int
    eps: float
    converged: bool
    eps_hist: np.ndarray
    h: np.ndarray | None = None


def si_solve(mask: np.ndarray, delta, nv: int, *, periodic_y: bool = False,
             cells_per_H: float | None = None, alpha: float = 1.0,
             drive: float = 1.0, wall_velocity=(0.0, 0.0), dy=None,
             tol: float = 1e-12, max_iter: int = 100000,
             return_h: bool = False) -> SIResult:
    """Run the paper's source iteration to the stop rule (FP64, CPU).

    ``delta`` is a scalar or a (ny, nx) field; ``cells_per_H`` defaults to ny.
    ``drive`` scales the pressure-gradient source (1: Poiseuille, 0: Couette);
    ``wall_velocity`` = (bottom, top) x velocities of the outer walls.
    ``dy`` = ny row heights in units of H (nonuniform rows), else uniform.
    ``tol < 0`` runs exactly ``max_iter`` iterations.
    """
    lib = _load()
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    ny, nx = m.shape
    if cells_per_H is None:
        cells_per_H = float(ny)
    d = np.ascontiguousarray(np.broadcast_to(np.asarray(delta, dtype=np.float64), (ny, nx))
                             if np.ndim(delta) else np.array([float(delta)]))
    field = int(np.ndim(delta) != 0)
    rho, u1, u2, tau, p12 = (np.zeros((ny, nx)) for _ in range(5))
    info = np.zeros(3)
    hist = np.zeros(max_iter)
    h = np.zeros((nv * nv, ny, nx)) if return_h else None
    dya = None if dy is None else np.ascontiguousarray(dy, dtype=np.float64)
    if dya is not None and dya.shape != (ny,):
        raise ValueError("dy needs one height per row")
    rc = lib.oracle_si_solve(nx, ny, _ptr(m), int(periodic_y), float(cells_per_H), _ptr(dya), nv,
                             _ptr(d), field, float(alpha), float(drive),
                             float(wall_velocity[0]), float(wall_velocity[1]),
                             float(tol), int(max_iter),
                             _ptr(rho), _ptr(u1), _ptr(u2), _ptr(tau), _ptr(p12),
                             _ptr(info), _ptr(hist), _ptr(h))
    if rc < 0:
        raise ValueError(f"oracle_si_solve rejected its input (rc={rc})")
    it = int(info[1])
    return SIResult(Q=float(info[0]), rho=rho, u1=u1, u2=u2, tau=tau, p12=p12,
                    iters=it, eps=float(info[2]), converged=(rc == 0),
                    eps_hist=hist[:it], h=h)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Host threads (OpenMP) of the oracle's next solves."""
    lib = _load()
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_num_threads.restype = None
    lib.oracle_set_num_threads(int(n))
