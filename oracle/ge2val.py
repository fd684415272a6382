"""Oracle of the two steps after the band reduction -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline leg
of ``bench.py`` may import this module.  It shares no code with the GPU
library.

The paper's singular-value pipeline (Section 2, and the GE2VAL runs of
Section 6.2) follows the band reduction GE2BND with BND2BD, band to
bidiagonal, and BD2VAL, bidiagonal to singular values.  It leaves the choice
of both methods open (any of the cited ones; its experiments use the
multi-threaded bulge chasing of PLASMA and LAPACK's bidiagonal QR).

* ``bnd2bd`` reduces an upper band matrix of bandwidth nb to upper bidiagonal
  form by two-sided Householder bulge chasing, one row per sweep: sweep k
  annihilates row k beyond its superdiagonal with a reflector from the right,
  which fills a triangle below the diagonal; a reflector from the left clears
  the first column of that triangle, which fills row k+1+... beyond the band
  one block further on; the sweep then chases this bulge down the band, a
  block of nb columns per step, until it falls off the end.  Only the first
  row or column of each bulge is cleared; the rest is cleared by the
  following sweeps.  The reflectors are applied to the whole matrix (every
  row, every column), so the result does not rest on any claim about where
  the fill lies; the tests check that every entry off the bidiagonal ends
  exactly zero.  ``windowed=True`` applies each reflector only to the rows
  or columns the sweep's structure says can be nonzero (rows rr..c+nb-1 for
  the right reflector of a step at column c, columns c..c+2nb-1 for the
  left one), which is what a fast implementation does.
* ``bd2val`` returns the singular values of the bidiagonal (d, e) in
  decreasing order: the definition, by LAPACK's SVD of the dense matrix.

Householder convention (LAPACK's): for x = (alpha, x2), beta = -sign(alpha)
||x||, tau = (beta - alpha) / beta, v = (1, x2 / (alpha - beta)); H = I - tau
v v^T maps x to beta e1; tau = 0 (H = I) when x2 = 0.

Parity status: pinned by ``tests/test_oracle_ge2val.py`` -- exact bidiagonal
structure of the dense result, singular values of the input band by LAPACK's
SVD, the Frobenius norm, the uniqueness of |d|, |e| for a reduction that
leaves the first column in place (an independent Golub-Kahan-Lanczos
recurrence started at e1), a band already bidiagonal, the closed-form
spectrum of the all-ones bidiagonal, diagonal and 2 x 2 cases.
"""
from __future__ import annotations

import numpy as np


def _householder(x):
    """(v, tau, beta) with (I - tau v v^T) x = beta e1 (LAPACK's convention)."""
    alpha = float(x[0])
    xnorm = float(np.linalg.norm(x[1:])) if x.shape[0] > 1 else 0.0
    v = np.zeros_like(x)
    v[0] = 1.0
    if xnorm == 0.0:
        return v, 0.0, alpha
    beta = -np.copysign(np.hypot(alpha, xnorm), alpha)
    tau = (beta - alpha) / beta
    v[1:] = x[1:] / (alpha - beta)
    return v, tau, beta


def upper_band(B, n, nb):
    """The n x n upper band part of B: entries (i, j) with 0 <= j - i <= nb."""
    A = np.array(B[:n, :n], dtype=np.float64)
    return np.triu(np.tril(A, nb))


def bnd2bd_dense(B, nb, windowed=False):
    """Bulge chasing on the upper band of the square B (bandwidth nb >= 1).
    Returns the whole final matrix (bidiagonal up to exact zeros)."""
    n = B.shape[0]
    A = upper_band(B, n, nb)
    for k in range(max(n - 2, 0)):
        t = 0
        while True:
            c = k + 1 + t * nb                 # first column of this step's block
            if c >= n:
                break
            rr = k if t == 0 else c - nb       # row whose entries beyond column c are cleared
            ce = min(c + nb, n)
            # right reflector: clear A[rr, c+1:ce], applied to the rows below rr
            v, tau, beta = _householder(A[rr, c:ce].copy())
            A[rr, c] = beta
            A[rr, c + 1:ce] = 0.0
            if tau != 0.0:
                r0, r1 = (rr + 1, ce) if windowed else (0, n)
                rows = [i for i in range(r0, r1) if i != rr]
                blk = A[rows, c:ce]
                w = blk @ v
                A[rows, c:ce] = blk - tau * np.outer(w, v)
            # left reflector: clear A[c+1:ce, c], applied to the columns right of c
            v, tau, beta = _householder(A[c:ce, c].copy())
            A[c, c] = beta
            A[c + 1:ce, c] = 0.0
            if tau != 0.0:
                c0, c1 = (c + 1, min(c + 2 * nb, n)) if windowed else (0, n)
                cols = [j for j in range(c0, c1) if j != c]
                blk = A[c:ce, cols]
                w = v @ blk
                A[c:ce, cols] = blk - tau * np.outer(v, w)
            t += 1
    return A


def bnd2bd(B, nb, windowed=True):
    """(d, e): diagonal and superdiagonal of the bidiagonal form of the upper
    band of the square B."""
    A = bnd2bd_dense(B, nb, windowed=windowed)
    return np.diag(A).copy(), np.diag(A, 1).copy()


def bd2val(d, e):
    """Singular values of the upper bidiagonal with diagonal d and
    superdiagonal e, in decreasing order."""
    n = len(d)
    if n == 0:
        return np.zeros(0)
    Bd = np.diag(np.asarray(d, dtype=np.float64))
    if n > 1:
        Bd += np.diag(np.asarray(e, dtype=np.float64)[:n - 1], 1)
    return np.linalg.svd(Bd, compute_uv=False)
