"""Python binding of the C ABI in ``include/dvm.h`` (ctypes).

Argument marshalling only: every step of the solver runs in ``libdvm.so``
(gfx950 HIP kernels).  The library must have been built (``build.py``); there
is no fallback -- importing this module without the library raises.
PyTorch, when present, only supplies the HIP stream the work is issued on.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdvm.so")

DVM_OK = 0
DVM_EINVAL = -1
DVM_ENOMEM = -2
DVM_EHIP = -3
DVM_ESTATE = -4
DVM_ENOCONV = -5
DVM_EDIVERGED = -6
DVM_FP64 = 0
DVM_FP32_REFINE = 1
DVM_SCHED_AUTO = 0
DVM_SCHED_SKEW = 1
DVM_SCHED_WRAP = 2
DVM_ACCEL_AUTO = 0
DVM_ACCEL_NONE = 1
DVM_ACCEL_GMRES = 2
STATUS_NAMES = {0: "running", 1: "converged", 2: "max_iter", 3: "diverged"}
SCHED_NAMES = {DVM_SCHED_SKEW: "skew", DVM_SCHED_WRAP: "wrap"}

EXPORTED = ("dvm_create", "dvm_set_geometry", "dvm_solve", "dvm_solve_warm",
            "dvm_flow_rate", "dvm_get_moments", "dvm_grad", "dvm_destroy",
            "dvm_last_error", "dvm_version", "dvm_profile", "dvm_launch_shape",
            "dvm_permeability", "dvm_set_driving", "dvm_set_row_heights",
            "dvm_get_moments_noalloc")


class DVMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class dvm_config(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_long), ("block_iters", ctypes.c_int),
                ("use_graphs", ctypes.c_int), ("vel_per_lane", ctypes.c_int),
                ("waves_per_block", ctypes.c_int), ("tune_cache", ctypes.c_char_p),
                ("profile", ctypes.c_int), ("schedule", ctypes.c_int),
                ("accel", ctypes.c_int), ("krylov_dim", ctypes.c_int), ("persistent", ctypes.c_int),
                ("krylov_deflate", ctypes.c_int), ("warm_extrapolate", ctypes.c_int)]


class dvm_prof(ctypes.Structure):
    _fields_ = [("sweep_ms", ctypes.c_double), ("n_sweeps", ctypes.c_long),
                ("updates", ctypes.c_double), ("other_ms", ctypes.c_double),
                ("sweep32_ms", ctypes.c_double), ("n_sweeps32", ctypes.c_long),
                ("updates32", ctypes.c_double), ("persistent_blocks", ctypes.c_long),
                ("persistent_iters", ctypes.c_long)]


class dvm_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_long), ("sweeps_fp64", ctypes.c_long),
                ("rel_change", ctypes.c_double), ("est_error", ctypes.c_double),
                ("status", ctypes.c_int), ("schedule", ctypes.c_int)]


# allocator hooks of dvm_create: alloc(bytes, ud) -> device pointer, free(ptr, ud)
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_lib = None


class TorchAllocator:
    """Allocator hooks that take a context's device buffers from torch's
    caching allocator (on the given device and stream, by default the current
    ones).  Keeps count of the bytes it holds for the library."""

    def __init__(self, device=None, stream=None):
        import torch
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        self.live = {}
        self.calls = 0

        def _alloc(nbytes, _ud):
            try:
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            except RuntimeError:
                return None          # the library reports DVM_ENOMEM
            self.live[ptr] = int(nbytes)
            self.calls += 1
            return ptr

        def _free(ptr, _ud):
            if ptr:
                torch.cuda.caching_allocator_delete(ptr)
                self.live.pop(ptr, None)

        self.alloc_fn = _ALLOC_FN(_alloc)
        self.free_fn = _FREE_FN(_free)

    @property
    def bytes_held(self) -> int:
        return sum(self.live.values())


def load_library(path: str = LIB_PATH):
    """Load libdvm.so; raises if it is missing (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with paper_1704_03126_amd/build.py")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.dvm_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, ctypes.c_int,
                               ctypes.POINTER(dvm_config), P, _ALLOC_FN, _FREE_FN, P]
    lib.dvm_set_geometry.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P,
                                     ctypes.c_int, ctypes.c_double]
    lib.dvm_solve.argtypes = [P, ctypes.c_int, P, ctypes.c_int, ctypes.c_double,
                              ctypes.POINTER(dvm_info)]
    lib.dvm_solve_warm.argtypes = lib.dvm_solve.argtypes
    lib.dvm_flow_rate.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)]
    lib.dvm_get_moments.argtypes = [P, ctypes.c_int, P, P, P, P, P]
    lib.dvm_get_moments_noalloc.argtypes = [P, ctypes.c_int, P, P, P, P, P]
    lib.dvm_grad.argtypes = [P, ctypes.c_int, P, ctypes.POINTER(ctypes.c_double)]
    lib.dvm_profile.argtypes = [P, ctypes.POINTER(dvm_prof)]
    IP = ctypes.POINTER(ctypes.c_int)
    lib.dvm_launch_shape.argtypes = [P, IP, IP, IP, IP]
    lib.dvm_set_row_heights.argtypes = [P, ctypes.c_int, P]
    lib.dvm_set_driving.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.dvm_permeability.argtypes = [ctypes.c_int, P, P, ctypes.c_double, P, P, P, P, P, P]
    lib.dvm_destroy.argtypes = [P]
    lib.dvm_destroy.restype = None
    lib.dvm_last_error.restype = ctypes.c_char_p
    lib.dvm_version.restype = ctypes.c_char_p
    for name in EXPORTED:
        getattr(lib, name)
    _lib = lib
    return lib


def _check(rc: int):
    if rc != DVM_OK:
        raise DVMError(rc, load_library().dvm_last_error().decode())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


@dataclass
class SolveInfo:
    iters: int
    sweeps_fp64: int
    rel_change: float
    est_error: float
    status: str
    schedule: str = ""


def permeability(delta, Q, porosity: float) -> dict:
    """Intrinsic permeability k_inf (Kn -> 0 limit of k_a), H*/H, and Kn*,
    k_a/k_inf per sample of a rarefaction sweep (dvm_permeability)."""
    lib = load_library()
    d = np.ascontiguousarray(delta, dtype=np.float64).ravel()
    q = np.ascontiguousarray(Q, dtype=np.float64).ravel()
    if d.shape != q.shape:
        raise ValueError("delta and Q must have the same length")
    k, h = ctypes.c_double(), ctypes.c_double()
    kns, rat, kn, ka = (np.zeros_like(d) for _ in range(4))
    _check(lib.dvm_permeability(len(d), _ptr(d), _ptr(q), float(porosity), ctypes.byref(k),
                                ctypes.byref(h), _ptr(kns), _ptr(rat), _ptr(kn), _ptr(ka)))
    return {"k_inf": k.value, "H_star": h.value, "Kn_star": kns, "ka_ratio": rat,
            "Kn": kn, "k_a": ka}


class Solver:
    """One context of the C ABI: n_instances problems on one velocity grid."""

    def __init__(self, nv: int, n_instances: int = 1, *, precision: int = DVM_FP64,
                 tol: float = 1e-8, max_iter: int = 200000, block_iters: int = 32,
                 use_graphs: bool = True, vel_per_lane: int = 0,
                 waves_per_block: int = 0, profile: bool = False, schedule: int = DVM_SCHED_AUTO,
                 accel: int = DVM_ACCEL_AUTO, krylov_dim: int = 0, tune_cache: str | None = None,
                 stream=None, allocator: TorchAllocator | None = None, persistent: bool = False,
                 krylov_deflate: int = 0, warm_extrapolate: bool = False):
        lib = load_library()
        tc = tune_cache.encode() if tune_cache else None
        cfg = dvm_config(precision, tol, max_iter, block_iters, int(use_graphs),
                         vel_per_lane, waves_per_block, tc, int(profile), int(schedule),
                         int(accel), int(krylov_dim), int(persistent), int(krylov_deflate),
                         int(warm_extrapolate))
        h = ctypes.c_void_p()
        s = stream if stream is not None else _current_stream()
        self.allocator = allocator          # kept alive until dvm_destroy
        if allocator is not None:
            fa, ff = allocator.alloc_fn, allocator.free_fn
        else:
            fa, ff = _ALLOC_FN(), _FREE_FN()
        _check(lib.dvm_create(ctypes.byref(h), nv, n_instances, ctypes.byref(cfg), s, fa, ff, None))
        self._h = h
        self._lib = lib
        self.epoch = 0              # bumped by every solve (autograd checks it)
        self.nv = nv
        self.n_instances = n_instances
        self.shapes = [None] * n_instances

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dvm_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def set_geometry(self, instance: int, mask, periodic_y: bool, cells_per_H: float):
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        ny, nx = m.shape
        _check(self._lib.dvm_set_geometry(self._h, instance, nx, ny, _ptr(m),
                                          int(periodic_y), float(cells_per_H)))
        self.shapes[instance] = (ny, nx)

    def _delta_arg(self, instance, delta):
        if instance >= 0:
            if np.ndim(delta) == 0:
                return np.array([float(delta)]), 0
            d = np.ascontiguousarray(delta, dtype=np.float64)
            if d.shape != self.shapes[instance]:
                raise ValueError("delta field shape does not match the geometry")
            return d, 1
        if all(np.ndim(d) == 0 for d in delta):
            return np.ascontiguousarray(np.asarray(delta, dtype=np.float64)), 0
        parts = [np.ascontiguousarray(np.broadcast_to(np.asarray(d, dtype=np.float64),
                                                      self.shapes[i])).ravel()
                 for i, d in enumerate(delta)]
        return np.ascontiguousarray(np.concatenate(parts)), 1

    def solve(self, instance: int, delta, alpha: float = 1.0, warm: bool = False,
              raise_on_noconv: bool = True):
        """Solve one instance (or all, instance -1) to the stop rule; returns
        its SolveInfo (a list for -1).  With raise_on_noconv False, instances
        that stop at max_iter or diverge do not raise: their status says so."""
        d, field = self._delta_arg(instance, delta)
        n = self.n_instances if instance < 0 else 1
        infos = (dvm_info * n)()
        fn = self._lib.dvm_solve_warm if warm else self._lib.dvm_solve
        self.epoch += 1
        rc = fn(self._h, instance, _ptr(d), field, float(alpha), infos)
        if rc != DVM_OK and not (rc in (DVM_ENOCONV, DVM_EDIVERGED) and not raise_on_noconv):
            _check(rc)
        out = [SolveInfo(i.iters, i.sweeps_fp64, i.rel_change, i.est_error,
                         STATUS_NAMES.get(i.status, str(i.status)),
                         SCHED_NAMES.get(i.schedule, str(i.schedule))) for i in infos]
        return out if instance < 0 else out[0]

    def set_row_heights(self, instance: int, dy=None):
        """Rows of unequal height (units of H, bottom row first); None:
        uniform rows of 1 / cells_per_H."""
        if dy is None:
            _check(self._lib.dvm_set_row_heights(self._h, instance, None))
            return
        ny, _ = self.shapes[instance]
        d = np.ascontiguousarray(dy, dtype=np.float64).ravel()
        if d.shape != (ny,):
            raise ValueError(f"need {ny} row heights")
        self._keep = getattr(self, "_keep", [])
        _check(self._lib.dvm_set_row_heights(self._h, instance, _ptr(d)))

    def set_driving(self, instance: int, pressure_gradient: float = 1.0, wall_velocity=(0.0, 0.0)):
        """Source of the flow: pressure-gradient factor (1: Poiseuille) and the
        x velocities (bottom, top) of the outer walls ((0, 1) with gradient 0:
        the Couette problem)."""
        _check(self._lib.dvm_set_driving(self._h, instance, float(pressure_gradient),
                                         float(wall_velocity[0]), float(wall_velocity[1])))

    def delta_sweep(self, instance: int, deltas, alpha: float = 1.0):
        """Solve one instance along a rarefaction sweep, each solve starting
        from the previous solution (from the state extrapolated in log(delta)
        through the last two when the Solver was built with
        warm_extrapolate=True); returns (Q per delta, SolveInfo per delta)."""
        Qs, infos = [], []
        for i, d in enumerate(deltas):
            infos.append(self.solve(instance, float(d), alpha, warm=i > 0))
            Qs.append(self.flow_rate(instance)[0])
        return np.array(Qs), infos

    def flow_rate(self, instance: int = 0):
        Q = ctypes.c_double()
        ka = ctypes.c_double()
        _check(self._lib.dvm_flow_rate(self._h, instance, ctypes.byref(Q), ctypes.byref(ka)))
        return Q.value, ka.value

    def moments(self, instance: int = 0, shear: bool = False):
        ny, nx = self.shapes[instance]
        out = {k: np.zeros((ny, nx)) for k in ("rho", "u1", "u2", "tau")}
        p12 = np.zeros((ny, nx)) if shear else None
        _check(self._lib.dvm_get_moments(self._h, instance, _ptr(out["rho"]), _ptr(out["u1"]),
                                         _ptr(out["u2"]), _ptr(out["tau"]), _ptr(p12)))
        if shear:
            out["p12"] = p12
        return out

    def moments_into(self, instance: int, rho=None, u1=None, u2=None, tau=None, p12=None):
        """dvm_get_moments_noalloc: the moments written into caller-owned
        device tensors (float64, ny x nx, contiguous; any may be None) on the
        context's stream, with no allocation."""
        ny, nx = self.shapes[instance]
        ptrs = []
        for t in (rho, u1, u2, tau, p12):
            if t is None:
                ptrs.append(None)
                continue
            if not (t.is_cuda and t.dtype.is_floating_point and t.element_size() == 8 and
                    t.is_contiguous() and t.numel() == ny * nx):
                raise ValueError("outputs must be contiguous float64 device tensors of the grid's size")
            ptrs.append(ctypes.c_void_p(t.data_ptr()))
        _check(self._lib.dvm_get_moments_noalloc(self._h, instance, *ptrs))

    def profile(self) -> dict:
        """Sweep timings since the last call (profile=True contexts): total
        ms, launch count and fluid updates of the FP64 and of the FP32 sweeps,
        and the ms of the other kernels of the plain FP64 iterations; in every
        context, the blocks run as one persistent launch and their
        iterations."""
        p = dvm_prof()
        _check(self._lib.dvm_profile(self._h, ctypes.byref(p)))
        return {f: getattr(p, f) for f, _ in dvm_prof._fields_}

    def launch_shape(self):
        """((V, G) of the FP64 sweep, (V, G) of the FP32 sweep); zeros while
        an autotuned context has not solved yet."""
        v = [ctypes.c_int() for _ in range(4)]
        _check(self._lib.dvm_launch_shape(self._h, *[ctypes.byref(x) for x in v]))
        return (v[0].value, v[1].value), (v[2].value, v[3].value)

    def grad(self, instance: int = 0):
        ny, nx = self.shapes[instance]
        g = np.zeros((ny, nx))
        ga = ctypes.c_double()
        _check(self._lib.dvm_grad(self._h, instance, _ptr(g), ctypes.byref(ga)))
        return g, ga.value


def version() -> str:
    return load_library().dvm_version().decode()
