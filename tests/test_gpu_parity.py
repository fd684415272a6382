"""GPU parity: the HIP path against the FP64 oracle, through the C ABI.

B is unique up to B -> D1 B D2 (signs), so the comparison is elementwise after
sign normalization, plus exact band structure and singular values.  Tolerance
(FP64 throughout): ||B~_gpu - B~_oracle||_F <= 50 n eps ||A||_F, the
backward-error scale of a product of O(n) Householder reflectors.
"""
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


def run_gpu(bb, A, nb, tree, variant, **opts):
    B, vt, plan = bb.band(torch.from_numpy(A), nb, tree, variant, watchdog_s=10.0, **opts)
    torch.cuda.synchronize()
    return B.cpu().numpy(), plan


def check_against_oracle(A, Bg, nb, tol_scale=50.0):
    m, n = A.shape
    assert oracle.band_violation(Bg, nb) == 0.0
    Bo, _ = oracle.band_reduce(A, nb)
    d = np.linalg.norm(oracle.sign_normalize(Bg, nb) - oracle.sign_normalize(Bo, nb))
    nA = np.linalg.norm(A)
    assert d <= tol_scale * n * EPS * nA, (d / nA, tol_scale * n * EPS)
    return d / nA


SHAPES = [
    (512, 512, 64),     # the small square workload: 8 x 8 tiles
    (256, 256, 32),
    (200, 130, 32),     # ragged in both dimensions
    (384, 128, 128),    # tall, 3 x 1 tiles (single QR step + nothing else)
    (640, 256, 128),    # 5 x 2 tiles of the nb = 128 kernels
    (330, 200, 64),     # ragged, several tiles
]


@pytest.mark.parametrize("m,n,nb", SHAPES)
@pytest.mark.parametrize("tree", ["flatts", "flattt", "greedy", "auto"])
@pytest.mark.parametrize("variant", ["bidiag", "rbidiag"])
def test_band_matches_oracle(bb, m, n, nb, tree, variant):
    A = workloads.gaussian(m, n, seed=1000 + m + n + nb)
    print("case", m, n, nb, tree, variant, flush=True)
    Bg, _ = run_gpu(bb, A, nb, tree, variant, sched="levels")
    check_against_oracle(A, Bg, nb)


@pytest.mark.parametrize("m,n,nb,tree,variant", [
    (512, 512, 64, "flatts", "bidiag"),
    (640, 256, 128, "greedy", "rbidiag"),
    (1024, 384, 128, "auto", "rbidiag"),
    (330, 200, 64, "auto", "bidiag"),
    (200, 130, 32, "flattt", "rbidiag"),
])
def test_persistent_equals_levels_bitwise(bb, m, n, nb, tree, variant):
    """Each task's arithmetic is fixed, so any valid schedule gives the same bits."""
    A = workloads.gaussian(m, n, seed=7 + m)
    print("case", m, n, nb, tree, variant, flush=True)
    B1, _ = run_gpu(bb, A, nb, tree, variant, sched="levels")
    B2, _ = run_gpu(bb, A, nb, tree, variant, sched="persistent")
    B3, _ = run_gpu(bb, A, nb, tree, variant, sched="persistent", workgroups=7)
    np.testing.assert_array_equal(B1, B2)
    np.testing.assert_array_equal(B1, B3)
    check_against_oracle(A, B2, nb)


def test_qr_only_is_r_factor(bb):
    A = workloads.gaussian(700, 300, seed=3)
    Bg, _ = run_gpu(bb, A, 64, "greedy", "qronly", sched="persistent")
    R = np.linalg.qr(A, mode="r")
    s1, s2 = np.sign(np.diag(Bg[:300])), np.sign(np.diag(R))
    np.testing.assert_allclose(s1[:, None] * Bg[:300], s2[:, None] * R, rtol=0,
                               atol=50 * 300 * EPS * np.linalg.norm(A))
    assert np.all(Bg[300:] == 0.0)


def test_zero_matrix_and_zero_columns(bb):
    Z = np.zeros((256, 192))
    Bg, _ = run_gpu(bb, Z, 64, "auto", "bidiag", sched="persistent")
    assert np.all(Bg == 0.0)
    A = workloads.gaussian(256, 192, seed=5)
    A[:, 70] = 0.0
    A[:, 130:140] = 0.0
    Bg, _ = run_gpu(bb, A, 64, "greedy", "bidiag", sched="persistent")
    check_against_oracle(A, Bg, 64)


def test_single_tile_and_tall_single_column(bb):
    for (m, n, nb) in [(64, 64, 64), (50, 20, 32), (1000, 100, 128), (129, 129, 128)]:
        A = workloads.gaussian(m, n, seed=m + n)
        print("case", m, n, nb, flush=True)
        Bg, _ = run_gpu(bb, A, nb, "greedy", "bidiag", sched="persistent")
        check_against_oracle(A, Bg, nb)


@pytest.mark.parametrize("variant,tree", [("rbidiag", "greedy"), ("rbidiag", "auto"),
                                          ("bidiag", "greedy")])
def test_tall_graded_full_size(bb, variant, tree):
    """The 32768 x 2048, nb = 128 workload: sigma(B) equals the prescribed s to
    the Weyl bound of an FP64 backward-stable reduction, and B is exactly banded."""
    cfg = workloads.CONFIGS["tall_graded"]
    A, s = workloads.graded(cfg["m"], cfg["n"], *cfg["seeds"], cfg["smin"])
    print("case tall_graded", variant, tree, flush=True)
    Bg, _ = run_gpu(bb, A, cfg["nb"], tree, variant, sched="persistent")
    n = cfg["n"]
    assert oracle.band_violation(Bg, cfg["nb"]) == 0.0
    sB = np.linalg.svd(Bg[:n], compute_uv=False)
    err = np.max(np.abs(sB - s))
    assert err <= 50 * n * EPS * np.linalg.norm(A), err


@pytest.mark.parametrize("m,n,nb,tree,opts", [
    (2048, 512, 64, "greedy", {}),                  # 32 x 8 tiles: switches at step 2
    (2048, 512, 64, "auto", {"switch_step": 5}),
    (1100, 300, 32, "flatts", {"delta": 3.0}),      # ragged
    (1500, 700, 128, "flattt", {"switch_step": 2}),
])
def test_three_step_matches_oracle(bb, m, n, nb, tree, opts):
    """The three-step reduction (Section 4.5) reaches the same band form."""
    A = workloads.gaussian(m, n, seed=4000 + m + n)
    print("case threestep", m, n, nb, tree, opts, flush=True)
    Bg, _ = run_gpu(bb, A, nb, tree, "threestep", sched="persistent", **opts)
    check_against_oracle(A, Bg, nb)
