"""GPU parity of the nb = 256 tile path (the tile size of the 16384 x 16384
workload) against the FP64 oracle.

At nb = 256 a panel streams its trailing column tiles (a 256 x 16 tile takes
half of a wave's registers) and an update unit covers a 128-column half of a
tile; these tests pin both against the oracle on every tree and variant, on
square, tall and ragged shapes, in both schedules and the mixed-precision
modes, and check the factors Q and P through bb_apply_q / bb_apply_p.  The
full 16384 x 16384 size is checked through properties that hold at any size
(exact band, Frobenius norm, probe vectors through Q and P).
"""
import functools

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
EPS32 = 2.0 ** -24
NB = 256


@pytest.fixture(scope="module")
def bb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1611_06892_amd as m
    m.lib()
    return m


@functools.lru_cache(maxsize=None)
def case(m, n, seed):
    """Input and the oracle's sign-normalized band form (B does not depend on
    the tree or the variant, so one oracle run serves them all)."""
    A = workloads.gaussian(m, n, seed=seed)
    Bo, _ = oracle.band_reduce(A, NB)
    return A, oracle.sign_normalize(Bo, NB)


def gpu_band(bb, A, tree, variant, **opts):
    B, _, _ = bb.band(torch.from_numpy(A), NB, tree, variant, watchdog_s=20.0, **opts)
    torch.cuda.synchronize()
    return B.cpu().numpy()


def rel_err(A, Ro, Bg):
    assert oracle.band_violation(Bg, NB) == 0.0
    return np.linalg.norm(oracle.sign_normalize(Bg, NB) - Ro) / np.linalg.norm(A)


@pytest.mark.parametrize("m,n", [(512, 256), (1024, 768), (1100, 700), (300, 260)])
@pytest.mark.parametrize("tree", ["flatts", "flattt", "greedy", "auto"])
@pytest.mark.parametrize("variant", ["bidiag", "rbidiag"])
def test_nb256_matches_oracle(bb, m, n, tree, variant):
    A, Ro = case(m, n, 2560 + m + n)
    print("case nb256", m, n, tree, variant, flush=True)
    e = rel_err(A, Ro, gpu_band(bb, A, tree, variant, sched="levels"))
    assert e <= 50 * n * EPS, e


@pytest.mark.parametrize("tree,variant", [("greedy", "rbidiag"), ("auto", "bidiag"),
                                          ("greedy", "bidiag"), ("flatts", "rbidiag")])
def test_nb256_square_2048(bb, tree, variant):
    A, Ro = case(2048, 2048, 2561)
    print("case nb256 2048^2", tree, variant, flush=True)
    e = rel_err(A, Ro, gpu_band(bb, A, tree, variant, sched="persistent"))
    assert e <= 50 * 2048 * EPS, e


@pytest.mark.parametrize("m,n,tree,variant", [(1024, 768, "greedy", "bidiag"),
                                              (1100, 700, "auto", "rbidiag")])
def test_nb256_persistent_equals_levels_bitwise(bb, m, n, tree, variant):
    A, Ro = case(m, n, 2560 + m + n)
    print("case nb256 schedules", m, n, tree, variant, flush=True)
    B1 = gpu_band(bb, A, tree, variant, sched="levels")
    B2 = gpu_band(bb, A, tree, variant, sched="persistent")
    B3 = gpu_band(bb, A, tree, variant, sched="persistent", workgroups=5)
    np.testing.assert_array_equal(B1, B2)
    np.testing.assert_array_equal(B1, B3)


@pytest.mark.parametrize("prec", ["f64_upd_f32", "f64_upd_split32"])
def test_nb256_mixed_precision(bb, prec):
    A, Ro = case(1024, 768, 2560 + 1024 + 768)
    print("case nb256", prec, flush=True)
    e = rel_err(A, Ro, gpu_band(bb, A, "greedy", "bidiag", prec=prec, sched="persistent"))
    assert e <= 50 * 768 * EPS32, e


def test_nb256_apply_q_p(bb):
    m, n = 1100, 700
    A, _ = case(m, n, 2560 + m + n)
    plan = bb.Plan(m, n, NB, "greedy", "rbidiag", watchdog_s=20.0)
    S = bb.to_colmajor(torch.from_numpy(A))
    vt, ws = plan.alloc()
    plan.execute(S, m, vt, ws)
    assert bb.poll_error(ws) == 0
    B = S.t()
    Eq = torch.eye(m, n, dtype=torch.float64, device="cuda").t().contiguous()
    assert bb.poll_error(plan.apply_q(Eq, m, n, vt)) == 0
    Ep = torch.eye(n, n, dtype=torch.float64, device="cuda").t().contiguous()
    assert bb.poll_error(plan.apply_p(Ep, n, n, vt)) == 0
    Q, P = Eq.t().cpu().numpy(), Ep.t().cpu().numpy()
    inv = oracle.invariants(A, B.cpu().numpy(), Q, P)
    print("nb256 invariants", inv, flush=True)
    assert max(inv.values()) <= 50 * n * EPS, inv
    np.testing.assert_array_equal(P[:NB, :NB], np.eye(NB))


def test_nb256_square_graded_full_size(bb):
    """16384 x 16384, s geometric 1 .. 1e-6, BiDiag Greedy: exact band,
    ||B||_F = ||s|| and 8 probe vectors ||A x - Q (B (P^T x))|| within the
    backward-error bound."""
    cfg = workloads.CONFIGS["square_graded"]
    m, n = cfg["m"], cfg["n"]
    Ad, s = workloads.graded_device(m, n, *cfg["seeds"], cfg["smin"])
    S = bb.to_colmajor(Ad)
    plan = bb.Plan(m, n, NB, "greedy", "bidiag", watchdog_s=60.0)
    vt, ws = plan.alloc()
    print("case nb256 16384^2 reduction", flush=True)
    plan.execute(S, m, vt, ws)
    assert bb.poll_error(ws) == 0
    B = S.t()
    i = torch.arange(m, device="cuda")[:, None]
    jj = torch.arange(n, device="cuda")[None, :]
    assert bool(torch.all(B[(jj < i) | (jj > i + NB)] == 0.0))
    nA = float(torch.linalg.norm(Ad))
    fro = abs(float(torch.linalg.norm(B)) - float(np.linalg.norm(s))) / float(np.linalg.norm(s))
    assert fro <= 50 * n * EPS, fro
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    X = torch.randn(n, 8, generator=gen, device="cuda", dtype=torch.float64)
    Y1 = Ad @ X
    Xs = X.t().contiguous()                       # column-major n x 8
    print("case nb256 16384^2 probes", flush=True)
    assert bb.poll_error(plan.apply_p(Xs, n, 8, vt, transpose=True)) == 0
    Z = B @ Xs.t()                                # B (P^T x)
    Zs = Z.t().contiguous()
    assert bb.poll_error(plan.apply_q(Zs, m, 8, vt)) == 0
    err = float(torch.linalg.norm(Y1 - Zs.t())) / (nA * float(torch.linalg.norm(X)))
    print("probe error", err, "fro", fro, flush=True)
    assert err <= 50 * n * EPS, err
