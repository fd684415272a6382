"""GPU test of bb_execute_noalloc, the entry point for callers that cannot
allocate device memory: its output must equal bb_execute's (the same kernels
and schedule, so the same bits) on two calls in a row, the second on a
smaller input, with the device's free memory unchanged by the calls; plans
whose workspace exceeds the library's array are rejected."""
import ctypes

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


def reduce_both(bb, A, nb, tree, variant):
    m, n = A.shape
    plan = bb.Plan(m, n, nb, tree, variant)
    S0 = bb.to_colmajor(torch.from_numpy(A))
    Sref, Snoa = S0.clone(), S0.clone()
    vt, ws = plan.alloc(S0.device)
    vt2 = torch.empty_like(vt)
    plan.execute(Sref, m, vt, ws)
    assert bb.poll_error(ws) == 0
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    print("noalloc", m, n, nb, tree, variant, flush=True)
    plan.execute_noalloc(Snoa, m, vt2)
    assert bb.poll_error(None) == 0
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
    return Sref, Snoa, vt, vt2


def test_noalloc_matches_execute_twice_second_smaller(bb):
    for (m, n, nb, tree, variant) in [(1100, 700, 64, "greedy", "rbidiag"),
                                      (530, 300, 32, "flatts", "bidiag")]:
        A = workloads.gaussian(m, n, seed=m + n)
        Sref, Snoa, vt, vt2 = reduce_both(bb, A, nb, tree, variant)
        assert torch.equal(Snoa, Sref)
        assert torch.equal(vt2, vt)
        B = Snoa.t().cpu().numpy()
        assert oracle.band_violation(B, nb) == 0.0
        Bo, _ = oracle.band_reduce(A, nb)
        d = np.linalg.norm(oracle.sign_normalize(B, nb) - oracle.sign_normalize(Bo, nb))
        assert d <= 50 * n * EPS * np.linalg.norm(A), d


def test_noalloc_rejects_a_plan_larger_than_its_array(bb):
    m, n = 6144, 2048
    plan = bb.Plan(m, n, 32, "greedy", "bidiag")
    vt, ws = plan.workspace()
    assert ws > (32 << 20)
    L = bb.lib()
    v8 = ctypes.c_void_p(8)
    assert L.bb_execute_noalloc(plan._h, v8, m, v8, vt, None) == 6
    assert L.bb_execute_noalloc(plan._h, v8, m - 1, v8, vt, None) == -3
