"""Band-bidiagonalization oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline leg
of ``bench.py`` may import this package.  The GPU library under
``paper_1611_06892_amd`` never imports it, and the two share no code.

Contents
--------
* ``band_reduce`` / ``rbidiag_reduce`` / ``form_q`` / ``form_p``: ctypes wrappers
  of ``band_oracle.c`` (plain unblocked FP64 Householder band reduction, the
  element-level form of the BiDiag sequence of Section 3.4 and of the
  R-BiDiag sequence of Section 3.5).
* ``sign_normalize``: maps any band form B to the representative with a
  non-negative diagonal and non-negative band edge.  B is unique only up to
  B -> D1 B D2 with D1, D2 = diag(+-1) and D2 = I on the first nb columns
  (block Golub-Kahan argument: A P = Q B and A^T Q = P B^T fix each block by a
  thin QR), so elementwise comparisons are made after this map.
* ``band_violation`` / ``invariants``: the checks every band form must pass.

Parity status: every function here is pinned by ``tests/test_oracle.py``
(hand-derived fixtures, library QR/SVD special cases, an independent block
Golub-Kahan recurrence, orthogonality and residual bounds).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "band_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile band_oracle.c with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        # -O3 with AVX2/FMA code generation for any x86-64-v3 host, and no
        # contraction of a*b+c into fused operations: the arithmetic is
        # exactly the source's, as at any optimization level
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        i64, dp = ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
        lib.oracle_band_reduce.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, dp, i64, dp]
        lib.oracle_band_reduce.restype = ctypes.c_int
        lib.oracle_rbidiag_reduce.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, dp, i64, dp,
                                              dp, i64]
        lib.oracle_rbidiag_reduce.restype = ctypes.c_int
        lib.oracle_form_q.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64]
        lib.oracle_form_q.restype = ctypes.c_int
        lib.oracle_form_p.argtypes = [i64, dp, i64, dp, dp, i64]
        lib.oracle_form_p.restype = ctypes.c_int
        lib.oracle_last_flops.argtypes = []
        lib.oracle_last_flops.restype = ctypes.c_double
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Reflectors:
    """Column reflectors (VQ, tauq) and row reflectors (WP, taup) of one run."""

    def __init__(self, m, n, nb, VQ, tauq, WP, taup):
        self.m, self.n, self.nb = m, n, nb
        self.VQ, self.tauq, self.WP, self.taup = VQ, tauq, WP, taup


def band_reduce(A: np.ndarray, nb: int):
    """BiDiag at element granularity (Section 3.4).  Returns (B, reflectors).

    A is m x n with m >= n; it is not modified.  B is m x n FP64 with exact
    zeros outside 0 <= j - i <= nb and in rows >= n.
    """
    lib = _load()
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    B = np.asfortranarray(A.copy())
    VQ = np.zeros((m, max(n, 1)), order="F")
    WP = np.zeros((max(n, 1), max(n, 1)), order="F")
    tauq = np.zeros(max(n, 1))
    taup = np.zeros(max(n, 1))
    rc = lib.oracle_band_reduce(m, n, nb, _ptr(B), max(m, 1), _ptr(VQ), max(m, 1),
                                _ptr(tauq), _ptr(WP), max(n, 1), _ptr(taup))
    if rc != 0:
        raise ValueError("oracle_band_reduce: invalid argument %d" % -rc)
    return B, Reflectors(m, n, nb, VQ, tauq, WP, taup)


def last_flops() -> float:
    """Flops counted by the last band_reduce call (3 per generated entry, 4 per
    entry touched by a dot+axpy)."""
    return _load().oracle_last_flops()


def num_threads() -> int:
    return _load().oracle_num_threads()


def rbidiag_reduce(A: np.ndarray, nb: int) -> np.ndarray:
    """R-BiDiag at element granularity (Section 3.5): QR of A, then the band
    reduction of the n x n factor R.  Returns B only."""
    lib = _load()
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    B = np.asfortranarray(A.copy())
    VQ = np.zeros((max(n, 1), max(n, 1)), order="F")
    WP = np.zeros((max(n, 1), max(n, 1)), order="F")
    R = np.zeros((max(n, 1), max(n, 1)), order="F")
    tauq = np.zeros(max(n, 1))
    taup = np.zeros(max(n, 1))
    rc = lib.oracle_rbidiag_reduce(m, n, nb, _ptr(B), max(m, 1), _ptr(VQ), max(n, 1),
                                   _ptr(tauq), _ptr(WP), max(n, 1), _ptr(taup), _ptr(R),
                                   max(n, 1))
    if rc != 0:
        raise ValueError("oracle_rbidiag_reduce: invalid argument %d" % -rc)
    return B


def form_q(refl: Reflectors, ncols: int | None = None) -> np.ndarray:
    """Q(:, :ncols) with Q = H_0 H_1 ... H_{n-1} (thin Q by default)."""
    lib = _load()
    m, n = refl.m, refl.n
    ncols = n if ncols is None else ncols
    Q = np.zeros((m, max(ncols, 1)), order="F")
    rc = lib.oracle_form_q(m, n, _ptr(refl.VQ), max(m, 1), _ptr(refl.tauq), ncols, _ptr(Q),
                           max(m, 1))
    if rc != 0:
        raise ValueError("oracle_form_q: invalid argument %d" % -rc)
    return Q[:, :ncols]


def form_p(refl: Reflectors) -> np.ndarray:
    """P = G_0 G_1 ... G_{n-1} (n x n)."""
    lib = _load()
    n = refl.n
    P = np.zeros((max(n, 1), max(n, 1)), order="F")
    lib.oracle_form_p(n, _ptr(refl.WP), max(n, 1), _ptr(refl.taup), _ptr(P), max(n, 1))
    return P[:n, :n]


def band_violation(B: np.ndarray, nb: int) -> float:
    """Largest |B(i,j)| outside the band 0 <= j - i <= nb (rows >= n included).
    Exactly 0.0 for a correct band form."""
    B = np.asarray(B)
    m, n = B.shape
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    outside = (j < i) | (j > i + nb)
    if not outside.any():
        return 0.0
    return float(np.max(np.abs(B[outside]))) if B.size else 0.0


def sign_vectors(B: np.ndarray, nb: int):
    """The +-1 vectors (s, t) of sign_normalize: t_c = +1 for c < nb; for
    i = 0..n-1: s_i = sgn(B_ii t_i), then t_{i+nb} = sgn(B_{i,i+nb} s_i) when
    i + nb < n (sgn(0) = +1).  With A = Q B P^T, also A = (Q diag(s))
    (diag(s) B diag(t)) (P diag(t))^T."""
    B = np.asarray(B, dtype=np.float64)
    n = B.shape[1]
    s = np.ones(n)
    t = np.ones(n)
    for i in range(n):
        s[i] = 1.0 if B[i, i] * t[i] >= 0 else -1.0
        if i + nb < n:
            t[i + nb] = 1.0 if B[i, i + nb] * s[i] >= 0 else -1.0
    return s, t


def sign_normalize(B: np.ndarray, nb: int) -> np.ndarray:
    """Representative of {D1 B D2} with B(i,i) >= 0 and B(i,i+nb) >= 0:
    diag(s) B[:n, :] diag(t) with (s, t) from sign_vectors (the n x n leading
    block)."""
    B = np.asarray(B, dtype=np.float64)
    n = B.shape[1]
    s, t = sign_vectors(B, nb)
    return (s[:, None] * B[:n, :]) * t[None, :]


def invariants(A: np.ndarray, B: np.ndarray, Q: np.ndarray, P: np.ndarray) -> dict:
    """Frobenius-norm checks for a band form with thin Q (m x n) and P (n x n):
    orthogonality of Q and P and the relative residual ||A - Q B[:n] P^T|| / ||A||."""
    n = A.shape[1]
    eye = np.eye(n)
    nA = np.linalg.norm(A)
    return {
        "orth_q": float(np.linalg.norm(Q.T @ Q - eye)),
        "orth_p": float(np.linalg.norm(P.T @ P - eye)),
        "residual": float(np.linalg.norm(A - Q @ B[:n, :] @ P.T) / (nA if nA > 0 else 1.0)),
    }
