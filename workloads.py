"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the band reduction itself: it only draws
matrices.  Both the GPU path and the oracle receive the arrays it returns.

Workloads (all FP64 generation; column-major arrays, m >= n):

* ``small_square``   512 x 512, iid N(0,1), seed 0; tile nb = 64 (8 x 8 tiles).
* ``tall_graded``    32768 x 2048, A = U diag(s) V^T with U the Q factor of a
                     seeded Gaussian (seed 1), V the Q factor of a seeded
                     Gaussian (seed 2), s_i = 10^(-8 i/(n-1)); nb = 128.
* ``square_graded``  16384 x 16384, the same recipe with seeds 3, 4 and
                     s geometric from 1 to 1e-6 (condition number 1e6); nb = 256.
* ``batch``          4096 matrices; m ~ U{64..1024}, then n ~ U{32..m}, then
                     entries N(0,1), in that order from one generator (seed 5).
* ``adjoint``        8192 x 1024 iid N(0,1) (seed 6), band weights W ~ N(0,1)
                     (seed 7); nb = 128.

The paper generated its test matrices with prescribed singular values
(LAPACK's LATMS, Section 6.1); ``graded`` is the stand-in: U diag(s) V^T with
known s, so sigma(B) can be checked against s directly.
"""
from __future__ import annotations

import numpy as np

CONFIGS = {
    "small_square": dict(m=512, n=512, nb=64, seed=0),
    "tall_graded": dict(m=32768, n=2048, nb=128, seeds=(1, 2), smin=1e-8),
    "square_graded": dict(m=16384, n=16384, nb=256, seeds=(3, 4), smin=1e-6),
    "batch": dict(count=4096, mlo=64, mhi=1024, nlo=32, seed=5),
    "adjoint": dict(m=8192, n=1024, nb=128, seed=6, wseed=7),
}


def gaussian(m: int, n: int, seed: int) -> np.ndarray:
    """m x n iid N(0,1), FP64, Fortran (column-major) order."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((m, n)))


def geometric_sigmas(n: int, smin: float) -> np.ndarray:
    """s_i = smin^(i/(n-1)), i = 0..n-1 (s_0 = 1, s_{n-1} = smin)."""
    if n == 1:
        return np.ones(1)
    return smin ** (np.arange(n) / (n - 1.0))


def orthonormal_columns(m: int, n: int, seed: int) -> np.ndarray:
    """Q factor (m x n, orthonormal columns) of a seeded m x n Gaussian."""
    q, _ = np.linalg.qr(gaussian(m, n, seed))
    return q


def graded(m: int, n: int, seed_u: int, seed_v: int, smin: float):
    """A = U diag(s) V^T with prescribed singular values s.  Returns (A, s)."""
    s = geometric_sigmas(n, smin)
    U = orthonormal_columns(m, n, seed_u)
    V = orthonormal_columns(n, n, seed_v)
    A = np.asfortranarray((U * s[None, :]) @ V.T)
    return A, s


def graded_device(m: int, n: int, seed_u: int, seed_v: int, smin: float, device="cuda"):
    """Same recipe as graded() for sizes where a host QR is too slow: the
    Gaussians come from a seeded torch generator on `device` and the Q factors
    from torch.linalg.qr there.  Returns (A as an m x n torch tensor, s)."""
    import torch
    s = geometric_sigmas(n, smin)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed_u)
    U, _ = torch.linalg.qr(torch.randn(m, n, generator=gen, device=device, dtype=torch.float64))
    gen.manual_seed(seed_v)
    V, _ = torch.linalg.qr(torch.randn(n, n, generator=gen, device=device, dtype=torch.float64))
    st = torch.from_numpy(s).to(device)
    A = (U * st[None, :]) @ V.t().contiguous()
    return A, s


def batch_shapes(count: int, seed: int, mlo: int = 64, mhi: int = 1024, nlo: int = 32):
    """Draw (m, n) pairs, then the entries, from one generator.  Returns a list
    of column-major FP64 matrices."""
    rng = np.random.default_rng(seed)
    mats = []
    for _ in range(count):
        m = int(rng.integers(mlo, mhi + 1))
        n = int(rng.integers(nlo, m + 1))
        mats.append(np.asfortranarray(rng.standard_normal((m, n))))
    return mats


def band_weights(n: int, nb: int, seed: int) -> np.ndarray:
    """n x n weights, N(0,1) inside the band 0 <= j - i <= nb, zero outside."""
    W = gaussian(n, n, seed)
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    W[(j < i) | (j > i + nb)] = 0.0
    return W


def flops_bidiag(m: int, n: int) -> float:
    """The operation count the paper reports GFLOP/s with, for both BiDiag
    and R-BiDiag (Section 6.2): 4 n^2 (m - n/3)."""
    return 4.0 * n * n * (m - n / 3.0)


def flops_rbidiag_actual(m: int, n: int) -> float:
    """Actual R-BiDiag count (Section 3.5): 2 n^2 (m + n)."""
    return 2.0 * n * n * (m + n)
