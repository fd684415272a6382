"""GPU parity of wide matrices (m < n), reduced as A^T (Section 3.6): the
result is the lower band form B = B'^T of A^T's upper band form B', and
A = Q B P^T with Q = P', P = Q'.  Checked against the oracle run on A^T,
and through the factors Q and P from bb_apply_q / bb_apply_p."""
import numpy as np
import pytest

import oracle
import workloads

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


def lower_band_violation(B, nb):
    return oracle.band_violation(np.ascontiguousarray(B.T), nb)


@pytest.mark.parametrize("m,n,nb", [(256, 512, 64), (130, 200, 32), (384, 1000, 128), (700, 1100, 256)])
@pytest.mark.parametrize("tree,variant", [("greedy", "rbidiag"), ("auto", "bidiag"), ("flatts", "bidiag")])
def test_wide_matches_oracle_of_transpose(bb, m, n, nb, tree, variant):
    A = workloads.gaussian(m, n, seed=3000 + m + n + nb)
    print("case wide", m, n, nb, tree, variant, flush=True)
    B, _, _ = bb.band(torch.from_numpy(A), nb, tree, variant, watchdog_s=20.0)
    Bg = B.cpu().numpy()
    assert lower_band_violation(Bg, nb) == 0.0
    Bo, _ = oracle.band_reduce(np.ascontiguousarray(A.T), nb)
    d = np.linalg.norm(oracle.sign_normalize(Bg.T, nb) - oracle.sign_normalize(Bo, nb))
    assert d <= 50 * m * EPS * np.linalg.norm(A), d


def test_wide_factors(bb):
    m, n, nb = 300, 700, 64
    A = workloads.gaussian(m, n, seed=31)
    plan = bb.Plan(m, n, nb, "greedy", "bidiag", watchdog_s=20.0)
    S = bb.to_colmajor(torch.from_numpy(A))
    vt, ws = plan.alloc()
    plan.execute(S, m, vt, ws)
    assert bb.poll_error(ws) == 0
    B = S.t().cpu().numpy()
    Eq = torch.eye(m, m, dtype=torch.float64, device="cuda").t().contiguous()
    assert bb.poll_error(plan.apply_q(Eq, m, m, vt)) == 0
    Ep = torch.eye(n, n, dtype=torch.float64, device="cuda").t().contiguous()
    assert bb.poll_error(plan.apply_p(Ep, n, n, vt)) == 0
    Q, P = Eq.t().cpu().numpy(), Ep.t().cpu().numpy()
    tol = 50 * n * EPS
    assert np.linalg.norm(Q.T @ Q - np.eye(m)) <= tol
    assert np.linalg.norm(P.T @ P - np.eye(n)) <= tol
    assert np.linalg.norm(A - Q @ B @ P.T) / np.linalg.norm(A) <= tol
    # Q = P' leaves the first nb rows alone (no LQ reflector of A^T touches them)
    np.testing.assert_array_equal(Q[:nb, :nb], np.eye(nb))
