"""Host helpers of the deflated GMRES restart (csrc/dvm_eig.h), compiled with
the host compiler and checked against numpy on the CPU.

The deflated restart keeps the harmonic Ritz vectors of a cycle's smallest
harmonic Ritz values (Morgan's GMRES-DR); what is checked here is what the
restart relies on: eigenvalues of small nonsymmetric matrices, the QR
factorisation of the kept block, and for a cycle of Arnoldi on a matrix with
a cluster of small eigenvalues the invariants of the deflated basis (P
orthonormal, the GMRES residual vector in its span, the harmonic Ritz values
it carries the smallest ones, and the Arnoldi relation Hb P_d = P Hn)."""
from __future__ import annotations

import ctypes
import shutil
import subprocess
from pathlib import Path

import numpy as np
import pytest

HERE = Path(__file__).resolve().parent


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    out = tmp_path_factory.mktemp("eig") / "eig_harness.so"
    subprocess.run([gxx, "-O2", "-Wall", "-Werror", "-shared", "-fPIC", "-o", str(out),
                    str(HERE / "eig_harness.cpp")], check=True)
    return ctypes.CDLL(str(out))


_dp = ctypes.POINTER(ctypes.c_double)


def _p(a):
    return a.ctypes.data_as(_dp)


def _f(a):
    return np.asfortranarray(a, dtype=np.float64)


def test_eigenvalues_match_numpy(lib):
    rng = np.random.default_rng(11)
    for n in (1, 2, 3, 4, 7, 16, 40, 64, 65):
        for t in range(12):
            A = rng.standard_normal((n, n))
            if t % 4 == 1:
                A = np.triu(A, -1)                       # already Hessenberg
            elif t % 4 == 2:
                A = A @ A.T + np.eye(n)                  # symmetric positive
            elif t % 4 == 3:
                A = np.diag(rng.uniform(-1, 1, n)) + 1e-3 * A   # near-diagonal
            re, im = np.zeros(n), np.zeros(n)
            assert lib.eig_values(_p(_f(A)), n, _p(re), _p(im)) == 0
            ev = re + 1j * im
            ref = np.linalg.eigvals(A)
            scale = max(1.0, np.abs(ref).max())
            # every computed value has a reference partner and vice versa
            assert max(np.abs(ref - e).min() for e in ev) < 1e-11 * scale
            assert max(np.abs(ev - r).min() for r in ref) < 1e-11 * scale


def test_small_qr(lib):
    rng = np.random.default_rng(12)
    for m, n in ((2, 1), (5, 4), (17, 16), (25, 24), (9, 5)):
        A = rng.standard_normal((m, n))
        Q, R = np.zeros(m * m), np.zeros(m * n)
        lib.eig_qr(_p(_f(A)), m, n, _p(Q), _p(R))
        Q, R = Q.reshape(m, m).T, R.reshape(n, m).T
        assert np.abs(Q @ R - A).max() < 1e-13
        assert np.abs(Q.T @ Q - np.eye(m)).max() < 1e-14
        assert np.abs(np.tril(R, -1)).max() == 0.0


def _arnoldi(n, k, seed):
    """One GMRES cycle of k Arnoldi steps on a nonnormal matrix with 20 small
    eigenvalues (the shape of a slowly contracting source iteration)."""
    rng = np.random.default_rng(seed)
    lam = np.concatenate([rng.uniform(0.002, 0.05, 20), rng.uniform(0.05, 1.5, n - 20)])
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    D = np.diag(np.exp(0.3 * rng.standard_normal(n)))
    A = D @ (Q * lam) @ Q.T @ np.linalg.inv(D)
    b = rng.standard_normal(n)
    V = np.zeros((n, k + 1))
    H = np.zeros((k + 1, k))
    beta = np.linalg.norm(b)
    V[:, 0] = b / beta
    for j in range(k):
        w = A @ V[:, j]
        for _ in range(2):
            h = V[:, :j + 1].T @ w
            H[:j + 1, j] += h
            w -= V[:, :j + 1] @ h
        H[j + 1, j] = np.linalg.norm(w)
        V[:, j + 1] = w / H[j + 1, j]
    c = np.zeros(k + 1)
    c[0] = beta
    y = np.linalg.lstsq(H, c, rcond=None)[0]
    return H, c - H @ y


@pytest.mark.parametrize("k,want", [(64, 16), (32, 8), (64, 24), (20, 4)])
def test_deflated_restart_invariants(lib, k, want):
    for seed in range(3):
        Hb, rho = _arnoldi(400, k, seed)
        P, Hn = np.zeros((k + 1) * (k + 1)), np.zeros((k + 1) * k)
        d = lib.eig_deflate(_p(_f(Hb)), k, _p(rho), want, _p(P), _p(Hn))
        assert d in (want, want + 1)             # a complex pair is kept whole
        P = P[:(k + 1) * (d + 1)].reshape(d + 1, k + 1).T
        Hn = Hn[:(d + 1) * d].reshape(d, d + 1).T
        assert np.abs(P.T @ P - np.eye(d + 1)).max() < 1e-13
        assert np.abs(P[k, :d]).max() == 0.0     # deflated columns live in V_k
        # the GMRES residual vector lies in the kept span
        assert np.linalg.norm(rho - P @ (P.T @ rho)) < 1e-12 * np.linalg.norm(rho)
        # Arnoldi relation of the restarted basis
        assert np.abs(Hb @ P[:k, :d] - P @ Hn).max() < 1e-10 * np.abs(Hb).max()
        # the kept subspace carries the d smallest harmonic Ritz values
        Hm = Hb[:k, :k]
        f = np.linalg.solve(Hm.T, np.eye(k)[:, -1])
        M = Hm + Hb[k, k - 1] ** 2 * np.outer(f, np.eye(k)[:, -1])
        th = np.sort(np.abs(np.linalg.eigvals(M)))[:d]
        B = np.linalg.lstsq(P[:k, :d], M @ P[:k, :d], rcond=None)[0]
        assert np.abs(np.sort(np.abs(np.linalg.eigvals(B))) - th).max() < 1e-10 * th.max()


def test_deflation_refused_without_invariance(lib):
    """Eigenvectors too ill-conditioned for the relation: a plain restart."""
    rng = np.random.default_rng(3)
    k = 64
    Hb = np.triu(rng.standard_normal((k + 1, k)), -1) * 0.1 + np.vstack([np.eye(k), np.zeros((1, k))])
    c = np.zeros(k + 1)
    c[0] = 1.0
    rho = c - Hb @ np.linalg.lstsq(Hb, c, rcond=None)[0]
    P, Hn = np.zeros((k + 1) * (k + 1)), np.zeros((k + 1) * k)
    assert lib.eig_deflate(_p(_f(Hb)), k, _p(rho), 16, _p(P), _p(Hn)) == 0
    assert lib.eig_deflate(_p(_f(Hb)), 1, _p(rho), 1, _p(P), _p(Hn)) == 0
