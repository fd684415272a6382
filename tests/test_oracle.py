"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

* Hand-derived band forms with exact values (tests/golden, Section 3.4 order and
  the Householder convention of the tile kernels of Section 3.2).
* Special cases that reduce to library routines: nb >= n is a QR factorization
  (numpy.linalg.qr), singular values are preserved (numpy.linalg.svd).
* An independent algorithm reaching the same band matrix: the block
  Golub-Kahan recurrence A P = Q B, A^T Q = P B^T with P's first block fixed
  to the identity, written here with library QR and full reorthogonalization.
  B is unique up to signs, so the sign-normalized results must agree.
* R-BiDiag (Section 3.5) reaches the same normalized band form as BiDiag.
* The leading term of the operation count at nb = 1 is 4mn^2 - 4n^3/3
  (Section 2, the GE2BD cost).
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import workloads

EPS = np.finfo(np.float64).eps
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_golden(name):
    nb, A, B, mode = None, [], [], None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line.startswith("nb"):
                nb = int(line.split()[1])
            elif line in ("A", "B"):
                mode = line
            else:
                (A if mode == "A" else B).append([float(x) for x in line.split()])
    return nb, np.array(A), np.array(B)


@pytest.mark.parametrize("name", ["hand_2x2_nb1.txt", "hand_3x3_nb1.txt",
                                  "hand_4x2_nb1_tall.txt"])
def test_hand_derived_fixtures(name):
    nb, A, Bexp = read_golden(name)
    B, _ = oracle.band_reduce(A, nb)
    np.testing.assert_allclose(B, Bexp, rtol=0, atol=8 * EPS * np.abs(A).max())


def block_golub_kahan(A, nb):
    """Independent route to the band form: block Golub-Kahan with P_0 = I[:, :nb].

    A P = Q B and A^T Q = P B^T determine, block by block, Q_k, B_kk (thin QR of
    A P_k - Q_{k-1} B_{k-1,k}) and P_{k+1}, B_{k,k+1} (thin QR of
    A^T Q_k - P_k B_kk^T), with every new block reorthogonalized twice against
    all previous blocks."""
    m, n = A.shape
    sizes = [min(nb, n - k) for k in range(0, n, nb)]
    offs = np.cumsum([0] + sizes)
    B = np.zeros((n, n))
    Qb, Pb = [], []
    P = np.zeros((n, sizes[0]))
    P[: sizes[0], : sizes[0]] = np.eye(sizes[0])
    Pb.append(P)
    prevQ, prevB = None, None
    for k, bk in enumerate(sizes):
        Y = A @ Pb[k]
        if prevQ is not None:
            Y = Y - prevQ @ prevB
        for _ in range(2):
            for Qo in Qb:
                Y = Y - Qo @ (Qo.T @ Y)
        Qk, Rk = np.linalg.qr(Y)
        Qb.append(Qk)
        B[offs[k]:offs[k + 1], offs[k]:offs[k + 1]] = Rk
        if k + 1 == len(sizes):
            break
        bn = sizes[k + 1]
        Z = A.T @ Qk - Pb[k] @ Rk.T
        for _ in range(2):
            for Po in Pb:
                Z = Z - Po @ (Po.T @ Z)
        Pq, Pr = np.linalg.qr(Z)
        Pn = Pq[:, :bn]
        Bk1 = Pr[:bn, :].T          # bk x bn, lower-trapezoidal
        Pb.append(Pn)
        B[offs[k]:offs[k + 1], offs[k + 1]:offs[k + 2]] = Bk1
        prevQ, prevB = Qk, Bk1
    return B


@pytest.mark.parametrize("m,n,nb", [(40, 24, 1), (37, 37, 1), (96, 32, 8), (70, 45, 16),
                                    (64, 64, 16), (130, 50, 7), (33, 20, 3)])
def test_matches_block_golub_kahan(m, n, nb):
    A = workloads.gaussian(m, n, seed=100 + m + n + nb)
    B, _ = oracle.band_reduce(A, nb)
    Bgk = block_golub_kahan(A, nb)
    d = np.linalg.norm(oracle.sign_normalize(B, nb) - oracle.sign_normalize(Bgk, nb))
    assert d / np.linalg.norm(A) <= 50 * n * EPS


@pytest.mark.parametrize("m,n,nb", [(8, 8, 1), (64, 64, 8), (100, 60, 16), (257, 130, 32),
                                    (50, 50, 64), (77, 31, 5), (1, 1, 1), (5, 1, 2)])
def test_band_structure_and_invariants(m, n, nb):
    A = workloads.gaussian(m, n, seed=m * 7 + n)
    B, refl = oracle.band_reduce(A, nb)
    assert oracle.band_violation(B, nb) == 0.0
    Q = oracle.form_q(refl)
    P = oracle.form_p(refl)
    inv = oracle.invariants(A, B, Q, P)
    tol = 50 * max(n, 1) * EPS
    assert inv["orth_q"] <= tol and inv["orth_p"] <= tol and inv["residual"] <= tol, inv
    # P leaves the first nb columns alone (the LQ steps never touch tile column 1).
    k = min(nb, n)
    np.testing.assert_array_equal(P[:, :k], np.eye(n)[:, :k])


@pytest.mark.parametrize("m,n,nb", [(60, 40, 4), (128, 128, 16), (90, 33, 10)])
def test_singular_values_preserved(m, n, nb):
    A = workloads.gaussian(m, n, seed=3 * m + n)
    B, _ = oracle.band_reduce(A, nb)
    sA = np.linalg.svd(A, compute_uv=False)
    sB = np.linalg.svd(B[:n], compute_uv=False)
    assert np.max(np.abs(sA - sB)) <= 50 * n * EPS * np.linalg.norm(A)


def test_prescribed_singular_values():
    A, s = workloads.graded(200, 64, 11, 12, 1e-8)
    B, _ = oracle.band_reduce(A, 8)
    sB = np.linalg.svd(B[:64], compute_uv=False)
    assert np.max(np.abs(sB - s)) <= 50 * 64 * EPS * np.linalg.norm(A)


@pytest.mark.parametrize("m,n", [(30, 12), (12, 12), (40, 1)])
def test_single_block_is_qr(m, n):
    """With nb >= n there is no LQ step: B[:n] is the R factor of A."""
    A = workloads.gaussian(m, n, seed=m + 5 * n)
    B, _ = oracle.band_reduce(A, n)
    R = np.linalg.qr(A, mode="r")
    Bn = B[:n]
    sb = np.sign(np.diag(Bn))
    sr = np.sign(np.diag(R))
    np.testing.assert_allclose(sb[:, None] * Bn, sr[:, None] * R, rtol=0,
                               atol=50 * n * EPS * np.linalg.norm(A))
    assert np.all(B[n:] == 0.0)


@pytest.mark.parametrize("m,n,nb", [(80, 32, 4), (64, 64, 8), (150, 40, 16), (45, 20, 3)])
def test_rbidiag_same_normalized_band(m, n, nb):
    A = workloads.gaussian(m, n, seed=2 * m + n + nb)
    B1, _ = oracle.band_reduce(A, nb)
    B2 = oracle.rbidiag_reduce(A, nb)
    assert oracle.band_violation(B2, nb) == 0.0
    d = np.linalg.norm(oracle.sign_normalize(B1, nb) - oracle.sign_normalize(B2, nb))
    assert d / np.linalg.norm(A) <= 50 * n * EPS


def test_flop_count_leading_term_nb1():
    m, n = 400, 300
    A = workloads.gaussian(m, n, seed=9)
    oracle.band_reduce(A, 1)
    f = oracle.last_flops()
    lead = 4.0 * m * n * n - 4.0 * n ** 3 / 3.0
    # The remainder is O(mn): relative gap O(1/n).
    assert abs(f - lead) / lead < 10.0 / n


def test_degenerate_inputs():
    # Zero matrix: every reflector is the identity (tau = 0) and B = 0.
    B, refl = oracle.band_reduce(np.zeros((9, 6)), 2)
    assert np.all(B == 0.0) and np.all(refl.tauq == 0.0) and np.all(refl.taup == 0.0)
    # Already in band form with a positive diagonal and positive band edge:
    # all tails are zero, nothing moves.
    n, nb = 7, 2
    D = np.triu(np.tril(np.arange(1.0, 50.0).reshape(7, 7), nb))
    B, _ = oracle.band_reduce(D, nb)
    np.testing.assert_array_equal(B, D)
    # A zero column inside the matrix keeps the invariants.
    A = workloads.gaussian(20, 10, seed=4)
    A[:, 3] = 0.0
    B, refl = oracle.band_reduce(A, 3)
    inv = oracle.invariants(A, B, oracle.form_q(refl), oracle.form_p(refl))
    assert max(inv.values()) <= 50 * 10 * EPS
    assert oracle.band_violation(B, 3) == 0.0


def test_invalid_arguments():
    with pytest.raises(ValueError):
        oracle.band_reduce(np.zeros((3, 5)), 2)      # m < n
    with pytest.raises(ValueError):
        oracle.band_reduce(np.zeros((5, 3)), 0)      # nb < 1


def test_sign_normalize_removes_sign_freedom():
    n, nb = 12, 3
    A = workloads.gaussian(20, n, seed=1)
    B, _ = oracle.band_reduce(A, nb)
    rng = np.random.default_rng(0)
    d1 = rng.choice([-1.0, 1.0], size=20)
    d2 = rng.choice([-1.0, 1.0], size=n)
    d2[:nb] = 1.0
    Bs = d1[:, None] * B * d2[None, :]
    np.testing.assert_array_equal(oracle.sign_normalize(B, nb), oracle.sign_normalize(Bs, nb))
    N = oracle.sign_normalize(B, nb)
    assert np.all(np.diag(N) >= 0)
    assert np.all(np.diag(N, nb) >= 0)


def test_thread_count_does_not_change_bits():
    code = ("import sys, hashlib; sys.path.insert(0, %r); import oracle, workloads;"
            "B,_ = oracle.band_reduce(workloads.gaussian(150, 90, 3), 10);"
            "sys.stdout.write(hashlib.sha256(B.tobytes()).hexdigest())") % \
        os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = []
    for t in ("1", "4"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        outs.append(subprocess.check_output([sys.executable, "-c", code], env=env))
    assert outs[0] == outs[1]


@pytest.mark.parametrize("m,n,nb", [(40, 24, 8), (30, 30, 6), (50, 20, 16), (36, 27, 8)])
def test_reference_gradient_matches_finite_differences(m, n, nb):
    """The autograd gradient of block Golub-Kahan (oracle/adjoint.py) against
    central differences of the unblocked C oracle, a different algorithm:
    L(A) = sum(W * B~(A)) with B~ the sign-normalized band form."""
    from oracle import adjoint
    rng = np.random.default_rng(m * n + nb)
    A = rng.standard_normal((m, n))
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    W = rng.standard_normal((n, n)) * ((j >= i) & (j <= i + nb))
    B0, _ = oracle.band_reduce(A, nb)
    Lref, G = adjoint.band_loss_gradient(A, W, nb, B0)

    def L(M):       # the loss on the oracle's own (raw, not normalized) band form
        return float(np.sum(W * oracle.band_reduce(M, nb)[0][:n]))

    assert abs(L(A) - Lref) <= 1e-10 * max(1.0, abs(Lref))
    h = 1e-6
    for d in range(4):
        E = rng.standard_normal((m, n))
        fd = (L(A + h * E) - L(A - h * E)) / (2 * h)
        an = float(np.sum(G * E))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def _exact_band(m, n, nb, seed):
    """An m x n matrix with random nonzero entries exactly on 0 <= j - i <= nb
    (rows >= n zero), the band form of Section 3.4, built entry by entry."""
    rng = np.random.default_rng(seed)
    B = np.zeros((m, n))
    for i in range(min(m, n)):
        for j in range(i, min(n, i + nb + 1)):
            B[i, j] = rng.uniform(1.0, 2.0) * rng.choice([-1.0, 1.0])
    return B


@pytest.mark.parametrize("m,n,nb", [(12, 9, 3), (9, 9, 1), (20, 7, 4)])
def test_band_violation_detects_each_outside_entry(m, n, nb):
    """band_violation must report exactly the one planted entry for every
    position outside the band (below the diagonal, beyond the band edge, in
    the rows >= n) and nothing for every position inside it (the diagonal and
    the band edge j - i = nb included)."""
    B = _exact_band(m, n, nb, seed=m + n + nb)
    assert oracle.band_violation(B, nb) == 0.0
    for i in range(m):
        for j in range(n):
            inside = i < n and 0 <= j - i <= nb
            C = B.copy()
            C[i, j] = 1e-300 if inside else 0.0
            if inside:
                assert oracle.band_violation(C, nb) == 0.0, (i, j)
                continue
            for v in (3.5, -0.25, 5e-324):
                C[i, j] = v
                assert oracle.band_violation(C, nb) == abs(v), (i, j, v)


def test_band_violation_named_positions():
    """The three positions a lax mask would miss: the subdiagonal (i, i-1),
    one past the band edge (i, i+nb+1) and a row below the n x n block."""
    m, n, nb = 10, 6, 2
    B = _exact_band(m, n, nb, seed=3)
    for (i, j), v in [((3, 2), 0.75), ((1, 1 + nb + 1), -2.0), ((n, 0), 1.25),
                      ((m - 1, n - 1), 4.0), ((n, n - 1), -3.0)]:
        C = B.copy()
        C[i, j] = v
        assert oracle.band_violation(C, nb) == abs(v)


@pytest.mark.parametrize("which", ["q", "p", "b"])
def test_invariants_reject_a_perturbed_factor(which):
    """invariants() must exceed the 50 n eps bound when one column of Q or P
    (or one band entry of B) is perturbed by far more than rounding: both the
    orthogonality and the residual measures see a column change."""
    m, n, nb = 30, 18, 4
    A = workloads.gaussian(m, n, seed=21)
    B, refl = oracle.band_reduce(A, nb)
    Q, P = oracle.form_q(refl), oracle.form_p(refl)
    tol = 50 * n * EPS
    base = oracle.invariants(A, B, Q, P)
    assert max(base.values()) <= tol
    rng = np.random.default_rng(5)
    if which == "q":
        Q = Q.copy()
        Q[:, 7] += 1e-9 * rng.standard_normal(m)
        inv = oracle.invariants(A, B, Q, P)
        assert inv["orth_q"] > tol and inv["residual"] > tol
        assert inv["orth_p"] <= tol
    elif which == "p":
        P = P.copy()
        P[:, 11] += 1e-9 * rng.standard_normal(n)
        inv = oracle.invariants(A, B, Q, P)
        assert inv["orth_p"] > tol and inv["residual"] > tol
        assert inv["orth_q"] <= tol
    else:
        B = B.copy()
        B[5, 5 + nb] *= 1 + 1e-9
        inv = oracle.invariants(A, B, Q, P)
        assert inv["residual"] > tol
        assert inv["orth_q"] <= tol and inv["orth_p"] <= tol
