"""GPU parity of the steps after the band reduction: BND2BD (bb_bnd2bd, band
to bidiagonal by bulge chasing) and BD2VAL (bb_bd2val, singular values of the
bidiagonal), and the whole GE2BND + BND2BD + BD2VAL pipeline.

* |d|, |e| of the device chase equal the oracle's element by element (the
  bidiagonal of a reduction that leaves the first column in place is unique
  up to signs) within 50 n eps ||B||_F, for tile-multiple and ragged n, every
  supported bandwidth class and the degenerate sizes, on the bands the band
  reduction produces; on an ill-conditioned random band, where those entries
  are sensitive to rounding, the singular values and the norm;
* the device bisection matches the oracle's singular values within
  50 n eps ||B||_2 (an absolute bound: bisection is accurate to a few
  eps ||B||);
* the pipeline returns the prescribed singular values of graded inputs, up to
  the full 16384 x 16384 square in the bench's launch configuration, both
  chained from the Python binding and as the C one-shot bb_ge2val;
* the chase's result does not depend on how many workgroups run a sweep
  (bit-identical for groups of 1 to 16);
* failure handling forced from the host: a watchdog of no clock ticks makes
  the launch end normally with BB_ETIMEOUT, through the one-shot pipeline too,
  and the next call is correct.
"""
import numpy as np
import pytest

import oracle
import workloads
from oracle import ge2val as og

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def bb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1611_06892_amd as m
    m.lib()
    return m


def colmajor(A):
    """(storage tensor, ld) of A as a column-major CUDA FP64 matrix."""
    return torch.from_numpy(np.ascontiguousarray(A.T)).cuda(), A.shape[0]


def band_input(kind, n, nb, seed):
    """The n x n band the band reduction leaves for an input of the paper's
    kinds: a tall N(0,1) matrix (m = 1.5 n), a square one, or a graded one
    (singular values 1 .. 1e-6), reduced by the oracle."""
    if kind == "graded":
        A, _ = workloads.graded(n, n, seed, seed + 1, 1e-6)
    else:
        A = workloads.gaussian(n + n // 2 if kind == "tall" else n, n, seed)
    B, _ = oracle.band_reduce(A, nb)
    return np.ascontiguousarray(B[:n, :n])


@pytest.mark.parametrize("n,nb,kind", [(1, 1, "tall"), (2, 3, "tall"), (3, 2, "square"), (9, 1, "tall"),
                                       (5, 2, "tall"), (64, 8, "square"), (100, 16, "tall"),
                                       (257, 32, "graded"), (300, 64, "tall"), (513, 64, "tall"),
                                       (640, 128, "tall"), (700, 256, "graded"), (1000, 32, "tall"),
                                       (50, 100, "square"), (129, 200, "tall"), (257, 256, "square"),
                                       (66, 65, "graded")])
def test_bnd2bd_matches_oracle(bb, n, nb, kind):
    print("case bnd2bd", n, nb, kind, flush=True)
    A = band_input(kind, n, nb, 7000 + n + nb)
    A[np.tril_indices(n, -1)] = 5.0          # below the band: must not be read
    S, ld = colmajor(A)
    d, e = bb.bnd2bd(S, ld, n, nb, watchdog_s=20.0)
    d, e = d.cpu().numpy(), e.cpu().numpy()
    do, eo = og.bnd2bd(A, nb)
    Bb = og.upper_band(A, n, nb)
    tol = 50 * n * EPS * np.linalg.norm(Bb)
    assert np.max(np.abs(np.abs(d) - np.abs(do)), initial=0.0) <= tol
    assert np.max(np.abs(np.abs(e) - np.abs(eo)), initial=0.0) <= tol
    # the input is read, never written
    assert np.array_equal(S.cpu().numpy(), np.ascontiguousarray(A.T))


@pytest.mark.parametrize("n,nb", [(300, 64), (700, 256)])
def test_bnd2bd_ill_conditioned_band_keeps_singular_values(bb, n, nb):
    """A random upper band is triangular and exponentially ill-conditioned:
    its bidiagonal entries are then sensitive to rounding (two correct
    orderings of the oracle already differ), but the singular values are
    not (Weyl), and neither is the Frobenius norm."""
    A = workloads.gaussian(n, n, seed=7100 + n)
    S, ld = colmajor(A)
    d, e = bb.bnd2bd(S, ld, n, nb, watchdog_s=20.0)
    Bb = og.upper_band(A, n, nb)
    s_ref = np.linalg.svd(Bb, compute_uv=False)
    s = og.bd2val(d.cpu().numpy(), e.cpu().numpy())
    tol = 50 * n * EPS * s_ref[0]
    assert np.max(np.abs(s - s_ref)) <= tol
    assert abs(np.sqrt(np.sum(d.cpu().numpy() ** 2) + np.sum(e.cpu().numpy() ** 2)) - np.linalg.norm(Bb)) <= tol


def test_bnd2bd_reads_a_leading_part_with_larger_ld(bb):
    m, n, nb = 700, 500, 64
    A = workloads.gaussian(m, n, seed=71)
    A[:n, :n] = band_input("tall", n, nb, 71)
    S, ld = colmajor(A)
    d, e = bb.bnd2bd(S, ld, n, nb, watchdog_s=20.0)
    do, eo = og.bnd2bd(A[:n, :n], nb)
    tol = 50 * n * EPS * np.linalg.norm(og.upper_band(A, n, nb))
    assert np.max(np.abs(np.abs(d.cpu().numpy()) - np.abs(do))) <= tol
    assert np.max(np.abs(np.abs(e.cpu().numpy()) - np.abs(eo))) <= tol


def test_bnd2bd_workspace_reused_and_too_small(bb):
    n, nb = 200, 32
    ws = torch.empty(bb.bnd2bd_workspace(n, nb), dtype=torch.uint8, device="cuda")
    for seed in (1, 2):
        A = band_input("square", n, nb, seed)
        S, ld = colmajor(A)
        d, e = bb.bnd2bd(S, ld, n, nb, ws=ws)
        do, eo = og.bnd2bd(A, nb)
        assert np.max(np.abs(np.abs(d.cpu().numpy()) - np.abs(do))) <= 50 * n * EPS * np.linalg.norm(A)
    small = ws[:-256]
    with pytest.raises(bb.BidiagError):
        bb.bnd2bd(S, ld, n, nb, ws=small)


@pytest.mark.parametrize("n", [1, 2, 3, 64, 1000, 4097])
def test_bd2val_matches_oracle(bb, n):
    rng = np.random.default_rng(11 + n)
    d = rng.standard_normal(n)
    e = rng.standard_normal(max(n - 1, 0))
    s = bb.bd2val(torch.from_numpy(d).cuda(), torch.from_numpy(e).cuda()).cpu().numpy()
    so = og.bd2val(d, e)
    assert np.max(np.abs(s - so)) <= 50 * n * EPS * so[0]
    assert np.all(np.diff(s) <= 0.0)


def test_bd2val_graded_and_structured(bb):
    n = 777
    # all-ones bidiagonal: 2 cos(k pi / (2n + 1))
    s = bb.bd2val(torch.ones(n, dtype=torch.float64).cuda(), torch.ones(n - 1, dtype=torch.float64).cuda())
    k = np.arange(1, n + 1)
    ref = 2.0 * np.cos(k * np.pi / (2 * n + 1))
    assert np.max(np.abs(s.cpu().numpy() - ref)) <= 50 * n * EPS * 2.0
    # graded diagonal, tiny coupling; zero singular values
    d = np.geomspace(1.0, 1e-12, n)
    d[::97] = 0.0
    e = 1e-3 * np.ones(n - 1)
    s = bb.bd2val(torch.from_numpy(d).cuda(), torch.from_numpy(e).cuda()).cpu().numpy()
    so = og.bd2val(d, e)
    assert np.max(np.abs(s - so)) <= 50 * n * EPS * so[0]


@pytest.mark.parametrize("m,n,nb,tree,variant", [(1024, 512, 64, "auto", "bidiag"),
                                                 (2000, 768, 128, "greedy", "rbidiag"),
                                                 (1300, 1300, 256, "auto", "bidiag"),
                                                 (400, 900, 32, "greedy", "bidiag")])
def test_ge2val_pipeline_returns_prescribed_singular_values(bb, m, n, nb, tree, variant):
    print("case ge2val", m, n, nb, tree, variant, flush=True)
    A, s = workloads.graded(max(m, n), min(m, n), 41, 42, 1e-6)
    if m < n:
        A = np.ascontiguousarray(A.T)          # a wide matrix has the same singular values
    sg = bb.ge2val(torch.from_numpy(A), nb, tree, variant, watchdog_s=20.0).cpu().numpy()
    ref = np.sort(s)[::-1]
    assert np.max(np.abs(sg - ref)) <= 50 * max(m, n) * EPS * ref[0]


def test_ge2val_band_stage_matches_oracle_on_the_device_band(bb):
    """BND2BD on the band the device reduction produced, against the oracle
    chase of that same band."""
    m, n, nb = 1500, 1100, 128
    A, _ = workloads.graded(m, n, 43, 44, 1e-6)
    B, _, _ = bb.band(torch.from_numpy(A), nb, "auto", "bidiag", watchdog_s=20.0)
    S = B.t()
    d, e = bb.bnd2bd(S, m, n, nb, watchdog_s=20.0)
    Bh = B.cpu().numpy()
    do, eo = og.bnd2bd(Bh[:n, :n], nb)
    tol = 50 * n * EPS * np.linalg.norm(Bh)
    assert np.max(np.abs(np.abs(d.cpu().numpy()) - np.abs(do))) <= tol
    assert np.max(np.abs(np.abs(e.cpu().numpy()) - np.abs(eo))) <= tol


@pytest.mark.parametrize("n,nb", [(700, 256), (640, 128), (1000, 96), (301, 65)])
def test_bnd2bd_result_does_not_depend_on_group_size(bb, n, nb):
    """For nb > 64 a sweep runs on a group of workgroups (rows and column
    chunks shared out, reflectors formed by every member): one workgroup a
    sweep (no group barriers), 2, 3, 8 and 16 give the same bits, and match the
    oracle."""
    print("case bnd2bd groups", n, nb, flush=True)
    A = band_input("tall", n, nb, 7300 + n)
    S, ld = colmajor(A)
    res = [bb.bnd2bd(S, ld, n, nb, watchdog_s=20.0, group=g) for g in (1, 2, 3, 8, 16)]
    for d, e in res[1:]:
        assert torch.equal(d, res[0][0]) and torch.equal(e, res[0][1])
    do, eo = og.bnd2bd(A, nb)
    tol = 50 * n * EPS * np.linalg.norm(og.upper_band(A, n, nb))
    assert np.max(np.abs(np.abs(res[0][0].cpu().numpy()) - np.abs(do))) <= tol
    assert np.max(np.abs(np.abs(res[0][1].cpu().numpy()) - np.abs(eo))) <= tol


def test_bnd2bd_group_out_of_range(bb):
    S = torch.zeros(10, 10, dtype=torch.float64, device="cuda")
    with pytest.raises(bb.BidiagError):
        bb.bnd2bd(S, 10, 10, 8, group=17)


@pytest.mark.parametrize("nb,tree", [(256, "auto"), (128, "greedy")])
def test_ge2val_full_size_square_graded(bb, nb, tree):
    """The 16384 x 16384 graded square (s geometric 1 .. 1e-6) through
    GE2BND, BND2BD and BD2VAL in the launch configuration the bench times:
    every singular value against the prescribed one within 50 n eps s_1
    (Weyl), and the bidiagonal's Frobenius norm against ||s||."""
    cfg = workloads.CONFIGS["square_graded"]
    m, n = cfg["m"], cfg["n"]
    Ad, s = workloads.graded_device(m, n, *cfg["seeds"], cfg["smin"])
    S = bb.to_colmajor(Ad)
    del Ad
    plan = bb.Plan(m, n, nb, tree, "bidiag", watchdog_s=60.0)
    vt, ws = plan.alloc()
    print("case ge2val 16384^2 nb", nb, tree, flush=True)
    plan.execute(S, m, vt, ws)
    assert bb.poll_error(ws) == 0
    del vt, ws
    d, e = bb.bnd2bd(S, m, n, nb, watchdog_s=60.0)
    sig = bb.bd2val(d, e).cpu().numpy()
    ref = np.sort(np.asarray(s))[::-1]
    tol = 50 * n * EPS * ref[0]
    assert np.max(np.abs(sig - ref)) <= tol
    fro = np.sqrt(np.sum(d.cpu().numpy() ** 2) + np.sum(e.cpu().numpy() ** 2))
    assert abs(fro - np.linalg.norm(ref)) <= tol * np.sqrt(n)


@pytest.mark.parametrize("n,nb", [(2000, 32), (1500, 128)])
def test_bnd2bd_watchdog_reports_timeout_and_recovers(bb, n, nb):
    """A watchdog of (almost) no clock ticks, set from the host: the first
    wait that is not satisfied at once reports BB_ETIMEOUT, every workgroup
    sees the error word and leaves (the launch ends normally), and the next
    call on the same workspace gives the oracle's bidiagonal."""
    print("case bnd2bd watchdog", n, nb, flush=True)
    A = band_input("square", n, nb, 7400 + n)
    S, ld = colmajor(A)
    ws = torch.empty(bb.bnd2bd_workspace(n, nb), dtype=torch.uint8, device="cuda")
    with pytest.raises(bb.BidiagError) as err:
        bb.bnd2bd(S, ld, n, nb, ws=ws, watchdog_s=1e-12)
    assert err.value.code == bb.poll_error(ws) == 3          # BB_ETIMEOUT
    d, e = bb.bnd2bd(S, ld, n, nb, ws=ws, watchdog_s=20.0)
    do, eo = og.bnd2bd(A, nb)
    tol = 50 * n * EPS * np.linalg.norm(og.upper_band(A, n, nb))
    assert np.max(np.abs(np.abs(d.cpu().numpy()) - np.abs(do))) <= tol
    assert np.max(np.abs(np.abs(e.cpu().numpy()) - np.abs(eo))) <= tol


@pytest.mark.parametrize("m,n,nb,tree,variant", [(1024, 512, 64, "auto", "bidiag"), (600, 900, 128, "greedy", "bidiag"),
                                                 (700, 700, 256, "auto", "bidiag"), (2000, 300, 32, "greedy", "rbidiag"),
                                                 (333, 500, 64, "greedy", "bidiag")])
def test_ge2val_oneshot_returns_prescribed_singular_values(bb, m, n, nb, tree, variant):
    """bb_ge2val (the C one-shot: GE2BND, BND2BD on the band or on the
    transpose of the lower band of a wide matrix, BD2VAL, one workspace)
    on graded inputs: the prescribed singular values."""
    print("case ge2val one-shot", m, n, nb, tree, variant, flush=True)
    A, s = workloads.graded(max(m, n), min(m, n), 51, 52, 1e-6)
    if m < n:
        A = np.ascontiguousarray(A.T)
    sg = bb.ge2val_oneshot(torch.from_numpy(A), nb, tree, variant, watchdog_s=20.0).cpu().numpy()
    ref = np.sort(s)[::-1]
    assert np.max(np.abs(sg - ref)) <= 50 * max(m, n) * EPS * ref[0]


def test_ge2val_oneshot_reports_a_failed_reduction(bb):
    """A band-reduction watchdog of no clock ticks, set from the host: the
    reduction reports BB_ETIMEOUT, the chase keeps that status and stops at
    its first wait, every launch ends normally, and bb_poll_error reports it;
    the next call gives the prescribed singular values."""
    m, n, nb = 1500, 1000, 64
    A, s = workloads.graded(m, n, 53, 54, 1e-6)
    with pytest.raises(bb.BidiagError) as err:
        bb.ge2val_oneshot(torch.from_numpy(A), nb, "greedy", "bidiag", watchdog_s=1e-12)
    assert err.value.code == 3          # BB_ETIMEOUT
    sg = bb.ge2val_oneshot(torch.from_numpy(A), nb, "greedy", "bidiag", watchdog_s=20.0).cpu().numpy()
    ref = np.sort(s)[::-1]
    assert np.max(np.abs(sg - ref)) <= 50 * m * EPS * ref[0]
