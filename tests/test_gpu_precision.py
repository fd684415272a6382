"""Precision extension: updates on FP32 matrix cores with FP64 panels.

Tolerance: the FP32 products carry a relative rounding error of order
eps32 = 2^-24 per entry, and each band form applies O(n) reflector blocks, so
the same backward-error argument as for FP64 gives
||B~_mixed - B~_oracle||_F <= 50 n eps32 ||A||_F (and the same Weyl bound on
singular values).  The split-FP32 form removes the operand rounding but keeps
the FP32 accumulation inside each matrix instruction, so it is held to the
same bound (measured: both land near 50 eps32, as FP64 lands near 50 eps64).
"""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -24


@pytest.fixture(scope="module")
def bb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1611_06892_amd as m
    m.lib()
    return m


def gpu_band(bb, A, nb, tree, variant, prec, **opts):
    B, _, _ = bb.band(torch.from_numpy(A), nb, tree, variant, prec=prec, watchdog_s=10.0, **opts)
    torch.cuda.synchronize()
    return B.cpu().numpy()


@pytest.mark.parametrize("m,n,nb", [(512, 512, 64), (640, 256, 128), (330, 200, 64), (200, 130, 32)])
@pytest.mark.parametrize("tree,variant", [("greedy", "bidiag"), ("auto", "rbidiag"),
                                          ("flatts", "bidiag")])
def test_mixed_precision_matches_oracle(bb, m, n, nb, tree, variant):
    A = workloads.gaussian(m, n, seed=500 + m + n)
    Bo, _ = oracle.band_reduce(A, nb)
    Ro = oracle.sign_normalize(Bo, nb)
    nA = np.linalg.norm(A)
    errs = {}
    for prec in ("f64", "f64_upd_f32", "f64_upd_split32"):
        Bg = gpu_band(bb, A, nb, tree, variant, prec, sched="levels")
        assert oracle.band_violation(Bg, nb) == 0.0, prec
        errs[prec] = np.linalg.norm(oracle.sign_normalize(Bg, nb) - Ro) / nA
    print("case", m, n, nb, tree, variant, errs, flush=True)
    assert errs["f64"] <= 50 * n * 2.0 ** -52
    assert errs["f64_upd_f32"] <= 50 * n * EPS32
    assert errs["f64_upd_split32"] <= 50 * n * EPS32


@pytest.mark.parametrize("prec", ["f64_upd_f32", "f64_upd_split32"])
def test_mixed_precision_schedules_agree_bitwise(bb, prec):
    A = workloads.gaussian(700, 300, seed=9)
    B1 = gpu_band(bb, A, 64, "greedy", "rbidiag", prec, sched="levels")
    B2 = gpu_band(bb, A, 64, "greedy", "rbidiag", prec, sched="persistent")
    np.testing.assert_array_equal(B1, B2)


def test_mixed_precision_singular_values_graded(bb):
    """Graded spectrum (1 .. 1e-6): the singular values of B stay within the
    FP32 Weyl bound of the prescribed ones."""
    A, s = workloads.graded(2048, 1024, 3, 4, 1e-6)
    for prec in ("f64_upd_f32", "f64_upd_split32"):
        Bg = gpu_band(bb, A, 128, "auto", "bidiag", prec)
        sB = np.linalg.svd(Bg[:1024], compute_uv=False)
        err = np.max(np.abs(sB - s))
        print(prec, "max |sigma - s| =", err, flush=True)
        assert err <= 50 * 1024 * EPS32 * np.linalg.norm(A)
