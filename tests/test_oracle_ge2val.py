"""Pins of the GE2VAL oracle (band -> bidiagonal -> singular values).

Each check rests on something other than the oracle's own formulas:

* the bulge chase is orthogonal: the singular values of (d, e) are those of
  the input band by LAPACK's SVD, and the Frobenius norm is kept;
* its result is exactly bidiagonal although every reflector is applied to
  the whole matrix (no structural assumption inside the oracle);
* no reflector touches the first column, so the bidiagonal is the one of
  the Golub-Kahan-Lanczos recurrence started at e1, unique up to signs: an
  independent recurrence (full reorthogonalisation) gives the same |d|, |e|;
* restricting each reflector to the rows/columns the structure allows
  changes nothing beyond rounding;
* a band of width 1 is already bidiagonal and is returned as it is;
* BD2VAL: the all-ones bidiagonal has singular values 2 cos(k pi / (2n+1)),
  a diagonal matrix has |d|, and a 2 x 2 matrix has sigma1 sigma2 = |d1 d2|
  and sigma1^2 + sigma2^2 = d1^2 + e1^2 + d2^2.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from oracle import ge2val  # noqa: E402

EPS = np.finfo(np.float64).eps
CASES = [(1, 1), (2, 1), (2, 3), (3, 2), (5, 2), (7, 3), (16, 4), (17, 4), (23, 5), (40, 8), (64, 7),
         (33, 32), (33, 40), (96, 16)]


def rand_band(n, nb, seed):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, n))
    B[np.tril_indices(n, -1)] = 99.0     # never read: only the upper band is the input
    return B


def band_part(B, nb):
    n = B.shape[0]
    return np.triu(np.tril(B, nb))


@pytest.mark.parametrize("n,nb", CASES)
def test_dense_result_is_exactly_bidiagonal(n, nb):
    A = ge2val.bnd2bd_dense(rand_band(n, nb, 1), nb)
    off = A - np.diag(np.diag(A)) - np.diag(np.diag(A, 1), 1)
    assert np.count_nonzero(off) == 0


@pytest.mark.parametrize("n,nb", CASES)
def test_singular_values_and_norm_are_kept(n, nb):
    B = rand_band(n, nb, 2)
    Bb = band_part(B, nb)
    d, e = ge2val.bnd2bd(B, nb)
    s_ref = np.linalg.svd(Bb, compute_uv=False)
    s = ge2val.bd2val(d, e)
    tol = 50 * n * EPS * max(s_ref[0], 1.0)
    assert np.max(np.abs(s - s_ref)) <= tol
    assert abs(np.sqrt(np.sum(d ** 2) + np.sum(e ** 2)) - np.linalg.norm(Bb)) <= tol


def golub_kahan_lanczos(B):
    """|d|, |e| of B = U Bd V^T with V e1 = e1 (Golub-Kahan-Lanczos from v1 = e1,
    full reorthogonalisation)."""
    n = B.shape[0]
    U = np.zeros((n, n))
    V = np.zeros((n, n))
    d = np.zeros(n)
    e = np.zeros(max(n - 1, 0))
    V[0, 0] = 1.0
    for i in range(n):
        u = B @ V[:, i] - (e[i - 1] * U[:, i - 1] if i > 0 else 0.0)
        for _ in range(2):
            u -= U[:, :i] @ (U[:, :i].T @ u)
        d[i] = np.linalg.norm(u)
        U[:, i] = u / d[i]
        if i < n - 1:
            v = B.T @ U[:, i] - d[i] * V[:, i]
            for _ in range(2):
                v -= V[:, :i + 1] @ (V[:, :i + 1].T @ v)
            e[i] = np.linalg.norm(v)
            V[:, i + 1] = v / e[i]
    return d, e


@pytest.mark.parametrize("n,nb", [(7, 2), (12, 3), (20, 5), (33, 8), (40, 4)])
def test_bidiagonal_matches_an_independent_lanczos_recurrence(n, nb):
    B = rand_band(n, nb, 3)
    d, e = ge2val.bnd2bd(B, nb)
    dl, el = golub_kahan_lanczos(band_part(B, nb))
    scale = np.linalg.norm(band_part(B, nb), 2)
    assert np.max(np.abs(np.abs(d) - dl)) <= 1e-10 * scale
    assert np.max(np.abs(np.abs(e) - el)) <= 1e-10 * scale


@pytest.mark.parametrize("n,nb", [(16, 4), (37, 6), (64, 16), (70, 9)])
def test_windowed_application_equals_the_dense_one(n, nb):
    B = rand_band(n, nb, 4)
    A = ge2val.bnd2bd_dense(B, nb, windowed=False)
    W = ge2val.bnd2bd_dense(B, nb, windowed=True)
    off = W - np.diag(np.diag(W)) - np.diag(np.diag(W, 1), 1)
    assert np.count_nonzero(off) == 0
    assert np.max(np.abs(A - W)) <= 1e-12 * np.linalg.norm(band_part(B, nb))


def test_width_one_band_is_returned_unchanged():
    B = rand_band(9, 1, 5)
    d, e = ge2val.bnd2bd(B, 1)
    assert np.array_equal(d, np.diag(B)) and np.array_equal(e, np.diag(B, 1))


@pytest.mark.parametrize("n", [1, 2, 5, 30, 200])
def test_bd2val_all_ones_closed_form(n):
    k = np.arange(1, n + 1)
    s = 2.0 * np.abs(np.cos(k * np.pi / (2 * n + 1)))
    assert np.max(np.abs(ge2val.bd2val(np.ones(n), np.ones(n - 1)) - np.sort(s)[::-1])) <= 1e-13


def test_bd2val_diagonal_and_two_by_two():
    d = np.array([3.0, -1.0, 0.5, -7.0, 0.0])
    assert np.array_equal(ge2val.bd2val(d, np.zeros(4)), np.sort(np.abs(d))[::-1])
    s = ge2val.bd2val(np.array([2.0, -3.0]), np.array([5.0]))
    assert abs(s[0] * s[1] - 6.0) <= 1e-13 * 6.0
    assert abs(s[0] ** 2 + s[1] ** 2 - 38.0) <= 1e-13 * 38.0
    assert s[0] >= s[1] >= 0.0
