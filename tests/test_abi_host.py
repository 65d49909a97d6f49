"""C-ABI checks that need no GPU: exports, argument validation, call order.

Every check in the library runs on the host before any device work, and a
context only touches the HIP runtime from its first solve on, so all of this
runs on a machine without a GPU.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1704_03126_amd.dvm as dvm
from paper_1704_03126_amd.geometry import plane_channel, rough_channel

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(dvm.LIB_PATH):
        from paper_1704_03126_amd.build import build
        build()
    return dvm.load_library()


def test_library_exports_every_declared_symbol(lib):
    header = open(os.path.join(ROOT, "include", "dvm.h")).read()
    declared = set(re.findall(r"\b(dvm_[a-z_]+)\s*\(", header))
    assert {"dvm_create", "dvm_set_geometry", "dvm_solve", "dvm_flow_rate",
            "dvm_grad"} <= declared
    for name in declared:
        assert hasattr(lib, name), name
    assert set(dvm.EXPORTED) == declared


def _ctx(lib, nv=8, n=1, **kw):
    cfg = dvm.dvm_config(kw.get("precision", 0), kw.get("tol", 1e-8), kw.get("max_iter", 1000),
                         kw.get("block_iters", 0), 1, kw.get("vel", 0), kw.get("waves", 0), None, 0,
                         kw.get("schedule", 0), 0, 0, kw.get("persistent", 0), kw.get("deflate", 0), kw.get("wx", 0))
    h = ctypes.c_void_p()
    rc = lib.dvm_create(ctypes.byref(h), nv, n, ctypes.byref(cfg), None,
                        kw.get("alloc", dvm._ALLOC_FN()), kw.get("free", dvm._FREE_FN()), None)
    return rc, h


def test_create_validates_arguments(lib):
    for nv in (3, 5, 2, 130):
        rc, _ = _ctx(lib, nv=nv)
        assert rc == dvm.DVM_EINVAL
    assert _ctx(lib, n=0)[0] == dvm.DVM_EINVAL
    assert _ctx(lib, precision=7)[0] == dvm.DVM_EINVAL
    assert _ctx(lib, tol=-1.0)[0] == dvm.DVM_EINVAL
    assert _ctx(lib, vel=3)[0] == dvm.DVM_EINVAL
    assert _ctx(lib, schedule=3)[0] == dvm.DVM_EINVAL
    assert _ctx(lib, persistent=2)[0] == dvm.DVM_EINVAL
    assert _ctx(lib, deflate=32)[0] == dvm.DVM_EINVAL
    assert _ctx(lib, wx=2)[0] == dvm.DVM_EINVAL
    for d in (-1, 8, 31):
        rc, h = _ctx(lib, deflate=d)
        assert rc == dvm.DVM_OK
        lib.dvm_destroy(h)
    rc, h = _ctx(lib, persistent=1)
    assert rc == dvm.DVM_OK
    lib.dvm_destroy(h)
    assert b"nv" in lib.dvm_last_error() or b"vel" in lib.dvm_last_error() or lib.dvm_last_error()
    rc, h = _ctx(lib)
    assert rc == dvm.DVM_OK
    lib.dvm_destroy(h)
    lib.dvm_destroy(None)


def test_create_allocator_hooks_come_in_pairs(lib):
    """Allocator hooks: both or neither; a context with hooks allocates
    nothing before its first solve (host-side set-up only)."""
    calls = []
    fa = dvm._ALLOC_FN(lambda n, ud: calls.append(n) or None)
    ff = dvm._FREE_FN(lambda p, ud: calls.append(p))
    assert _ctx(lib, alloc=fa)[0] == dvm.DVM_EINVAL
    assert b"alloc" in lib.dvm_last_error()
    assert _ctx(lib, free=ff)[0] == dvm.DVM_EINVAL
    rc, h = _ctx(lib, alloc=fa, free=ff)
    assert rc == dvm.DVM_OK
    m = np.zeros((8, 8), dtype=np.uint8)
    assert lib.dvm_set_geometry(h, 0, 8, 8, m.ctypes.data_as(ctypes.c_void_p), 0, 8.0) == 0
    lib.dvm_destroy(h)
    assert calls == []


def _set(lib, h, inst, mask, periodic_y=0, cph=None):
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    ny, nx = m.shape
    return lib.dvm_set_geometry(h, inst, nx, ny, m.ctypes.data_as(ctypes.c_void_p),
                                periodic_y, float(cph or ny))


def test_set_geometry_validation(lib):
    rc, h = _ctx(lib, n=2)
    assert rc == 0
    try:
        assert _set(lib, h, 0, plane_channel(16).mask) == 0
        assert _set(lib, h, 1, rough_channel(16, 12, 2, 8).mask) == 0
        assert _set(lib, h, 2, plane_channel(16).mask) == dvm.DVM_EINVAL      # index
        assert _set(lib, h, 0, np.zeros((16, 3), np.uint8)) == dvm.DVM_EINVAL  # nx 3
        assert _set(lib, h, 0, np.zeros((3, 8), np.uint8)) == dvm.DVM_EINVAL   # ny 3
        assert _set(lib, h, 0, np.full((8, 8), 2, np.uint8)) == dvm.DVM_EINVAL
        assert _set(lib, h, 0, np.ones((8, 8), np.uint8)) == dvm.DVM_EINVAL    # no fluid
        blocked = np.zeros((8, 8), np.uint8)
        blocked[:, 3] = 1                                                  # no flow path
        assert _set(lib, h, 0, blocked) == dvm.DVM_EINVAL
        assert b"wrap" in lib.dvm_last_error()
        pocket = np.zeros((10, 10), np.uint8)
        pocket[2:7, 2] = pocket[2:7, 6] = pocket[2, 2:7] = pocket[6, 2:7] = 1
        assert _set(lib, h, 0, pocket) == dvm.DVM_EINVAL                  # enclosed pore
        m = np.ascontiguousarray(plane_channel(8).mask)
        assert lib.dvm_set_geometry(h, 0, 1, 8, m.ctypes.data_as(ctypes.c_void_p), 0, -1.0) == dvm.DVM_EINVAL
        assert lib.dvm_set_geometry(h, 0, 1, 8, None, 0, 8.0) == dvm.DVM_EINVAL
    finally:
        lib.dvm_destroy(h)


def test_call_order_and_solve_arguments(lib):
    rc, h = _ctx(lib, n=2)
    d = np.array([1.0])
    info = dvm.dvm_info()
    dp = d.ctypes.data_as(ctypes.c_void_p)
    try:
        # no geometry yet
        assert lib.dvm_solve(h, 0, dp, 0, 1.0, ctypes.byref(info)) == dvm.DVM_ESTATE
        q = ctypes.c_double()
        assert lib.dvm_flow_rate(h, 0, ctypes.byref(q), None) == dvm.DVM_ESTATE
        assert _set(lib, h, 0, plane_channel(16).mask) == 0
        # bad arguments are rejected before any device work
        assert lib.dvm_solve(h, 0, dp, 0, 0.0, ctypes.byref(info)) == dvm.DVM_EINVAL
        assert lib.dvm_solve(h, 0, dp, 0, 1.5, ctypes.byref(info)) == dvm.DVM_EINVAL
        assert lib.dvm_solve(h, 0, None, 0, 1.0, ctypes.byref(info)) == dvm.DVM_EINVAL
        assert lib.dvm_solve(h, 5, dp, 0, 1.0, ctypes.byref(info)) == dvm.DVM_EINVAL
        for bad in (np.nan, -1.0, np.inf):
            b = np.array([bad])
            assert lib.dvm_solve(h, 0, b.ctypes.data_as(ctypes.c_void_p), 0, 1.0,
                                 ctypes.byref(info)) == dvm.DVM_EINVAL
        f = np.full((16, 1), 1.0)
        f[3, 0] = np.nan
        assert lib.dvm_solve(h, 0, f.ctypes.data_as(ctypes.c_void_p), 1, 1.0,
                             ctypes.byref(info)) == dvm.DVM_EINVAL
        # batched solve needs every instance described
        assert lib.dvm_solve(h, -1, dp, 0, 1.0, ctypes.byref(info)) == dvm.DVM_ESTATE
        assert lib.dvm_grad(h, 0, None, None) == dvm.DVM_ESTATE   # not solved yet
    finally:
        lib.dvm_destroy(h)


def test_driving_validation(lib):
    from paper_1704_03126_amd.geometry import porous_discs
    rc, h = _ctx(lib, n=2)
    d = np.array([1.0])
    dp = d.ctypes.data_as(ctypes.c_void_p)
    info = dvm.dvm_info()
    try:
        assert lib.dvm_set_driving(h, 2, 1.0, 0.0, 0.0) == dvm.DVM_EINVAL
        assert lib.dvm_set_driving(h, -1, 1.0, 0.0, 0.0) == dvm.DVM_EINVAL
        for bad in ((np.nan, 0.0, 0.0), (1.0, np.inf, 0.0), (1.0, 0.0, -np.inf)):
            assert lib.dvm_set_driving(h, 0, *bad) == dvm.DVM_EINVAL
        # driving set before the geometry is kept; a periodic cell cannot
        # have sliding walls (rejected before any device work)
        assert lib.dvm_set_driving(h, 1, 0.0, 0.0, 1.0) == 0
        g = porous_discs(16, 0.7, 3)
        assert _set(lib, h, 1, g.mask, periodic_y=1) == 0
        assert lib.dvm_solve(h, 1, dp, 0, 1.0, ctypes.byref(info)) == dvm.DVM_EINVAL
        assert b"sliding walls" in lib.dvm_last_error()
    finally:
        lib.dvm_destroy(h)


def test_row_heights_validation(lib):
    rc, h = _ctx(lib, n=1)
    try:
        dy = np.full(16, 1 / 16)
        dp = dy.ctypes.data_as(ctypes.c_void_p)
        assert lib.dvm_set_row_heights(h, 0, dp) == dvm.DVM_ESTATE      # no geometry yet
        assert _set(lib, h, 0, plane_channel(16).mask) == 0
        assert lib.dvm_set_row_heights(h, 1, dp) == dvm.DVM_EINVAL
        for bad in (0.0, -0.1, np.nan, np.inf):
            b = dy.copy()
            b[5] = bad
            assert lib.dvm_set_row_heights(h, 0, b.ctypes.data_as(ctypes.c_void_p)) == dvm.DVM_EINVAL
        assert lib.dvm_set_row_heights(h, 0, dp) == 0
        assert lib.dvm_set_row_heights(h, 0, None) == 0
    finally:
        lib.dvm_destroy(h)


def test_python_binding_fails_loudly_without_library(tmp_path):
    with pytest.raises(ImportError):
        dvm.load_library.__wrapped__ if hasattr(dvm.load_library, "__wrapped__") else None
        saved = dvm._lib
        dvm._lib = None
        try:
            dvm.load_library(str(tmp_path / "missing.so"))
        finally:
            dvm._lib = saved
