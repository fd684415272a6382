"""GPU tests of batched reductions (bb_batch_*): many independent matrices of
different sizes, tile sizes, trees and variants in one persistent launch
(tile sizes 32 to 128 share it; nb = 256 runs in a second).

Every matrix is checked against the FP64 oracle (sign-normalized B, exact
band), and against the same matrix reduced alone: a task computes the same
bits whatever else runs beside it, so the batched and single results must be
identical.
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


def mixed_batch(count, seed, mhi=400):
    rng = np.random.default_rng(seed)
    mats, nbs, trees, variants = [], [], [], []
    for _ in range(count):
        m = int(rng.integers(16, mhi + 1))
        n = int(rng.integers(8, m + 1))
        mats.append(np.asfortranarray(rng.standard_normal((m, n))))
        nbs.append(int(rng.choice([32, 64, 128])))
        trees.append(str(rng.choice(["flatts", "flattt", "greedy", "auto"])))
        variants.append(str(rng.choice(["bidiag", "rbidiag"])))
    return mats, nbs, trees, variants


def run_batch(bb, mats, **kw):
    plan = bb.BatchPlan([A.shape for A in mats], watchdog_s=20.0, **kw)
    buf, ptrs, ldas, offs = bb.pack_batch(mats)
    vt, ws = plan.alloc()
    plan.execute(ptrs, ldas, vt, ws)
    assert plan.poll_error(ws) == 0
    torch.cuda.synchronize()
    Bs = [bb.unpack(buf, offs, plan.shapes, i).cpu().numpy() for i in range(len(mats))]
    return plan, Bs


def test_mixed_batch_matches_oracle_and_single_runs(bb):
    mats, nbs, trees, variants = mixed_batch(40, seed=3)
    print("batch of", len(mats), flush=True)
    plan, Bs = run_batch(bb, mats, nb=nbs, tree=trees, variant=variants)
    for i, (A, B) in enumerate(zip(mats, Bs)):
        m, n = A.shape
        info = plan.info(i)
        assert (info["nb"], info["tree"], info["variant"]) == (nbs[i], trees[i], variants[i])
        assert oracle.band_violation(B, nbs[i]) == 0.0, i
        Bo, _ = oracle.band_reduce(A, nbs[i])
        d = np.linalg.norm(oracle.sign_normalize(B, nbs[i]) - oracle.sign_normalize(Bo, nbs[i]))
        assert d <= 50 * n * EPS * np.linalg.norm(A), (i, m, n, d)
    for i in (0, 7, 19, 39):
        print("single", i, mats[i].shape, nbs[i], trees[i], variants[i], flush=True)
        Bsingle, _, _ = bb.band(torch.from_numpy(mats[i]), nbs[i], trees[i], variants[i])
        assert np.array_equal(Bsingle.cpu().numpy(), Bs[i]), i


def test_tuned_batch_of_the_batch_recipe(bb):
    """The batch recipe (m ~ U{64..1024}, n ~ U{32..m}), 48 matrices, with the
    tuned (nb, tree, variant) per size class; a sample checked against the
    oracle, every matrix against its prescribed band structure and its
    Frobenius norm (orthogonal invariance)."""
    mats = workloads.batch_shapes(48, seed=5)
    print("tuned batch of", len(mats), flush=True)
    plan, Bs = run_batch(bb, mats)
    for i, (A, B) in enumerate(zip(mats, Bs)):
        nb = plan.info(i)["nb"]
        assert plan.info(i)["nb"] == bb.tuned_config(*A.shape)[0]
        assert oracle.band_violation(B, nb) == 0.0
        nA = np.linalg.norm(A)
        assert abs(np.linalg.norm(B) - nA) <= 50 * A.shape[1] * EPS * nA
    for i in range(0, 48, 12):
        A, B = mats[i], Bs[i]
        nb = plan.info(i)["nb"]
        Bo, _ = oracle.band_reduce(A, nb)
        d = np.linalg.norm(oracle.sign_normalize(B, nb) - oracle.sign_normalize(Bo, nb))
        assert d <= 50 * A.shape[1] * EPS * np.linalg.norm(A), (i, A.shape, d)


def size_class(m, n):
    """The tuner's size class of an m x n matrix: row range and aspect
    1000 n / m (the edges of the offline tuner)."""
    m_edges, r_edges = [64, 192, 384, 640, 1025], [0, 250, 500, 1000]
    ci = next(c for c in range(4) if m_edges[c] <= m < m_edges[c + 1])
    a = 1000.0 * n / m
    ri = next(r for r in range(3) if r_edges[r] < a <= r_edges[r + 1])
    return ci, ri


def test_full_batch_recipe_per_class_oracle_sample(bb):
    """The whole batch recipe, 4096 matrices (m ~ U{64..1024}, n ~ U{32..m},
    seed 5) in the launches of one plan with the tuned (nb, tree, variant):
    every matrix exact band and Frobenius norm; the first two matrices of
    each of the twelve size classes against the oracle."""
    cfg = workloads.CONFIGS["batch"]
    mats = workloads.batch_shapes(cfg["count"], cfg["seed"], cfg["mlo"], cfg["mhi"], cfg["nlo"])
    print("full batch of", len(mats), flush=True)
    plan, Bs = run_batch(bb, mats)
    picked = {}
    for i, (A, B) in enumerate(zip(mats, Bs)):
        nb = plan.info(i)["nb"]
        assert oracle.band_violation(B, nb) == 0.0, i
        nA = np.linalg.norm(A)
        assert abs(np.linalg.norm(B) - nA) <= 50 * A.shape[1] * EPS * nA, i
        picked.setdefault(size_class(*A.shape), [])
        if len(picked[size_class(*A.shape)]) < 2:
            picked[size_class(*A.shape)].append(i)
    assert len(picked) == 12
    for cls, idx in sorted(picked.items()):
        for i in idx:
            A, B = mats[i], Bs[i]
            nb = plan.info(i)["nb"]
            print("class", cls, "matrix", i, A.shape, "nb", nb, flush=True)
            Bo, _ = oracle.band_reduce(A, nb)
            d = np.linalg.norm(oracle.sign_normalize(B, nb) - oracle.sign_normalize(Bo, nb))
            assert d <= 50 * A.shape[1] * EPS * np.linalg.norm(A), (cls, i, A.shape, d)


def test_batch_reuse_and_timing(bb):
    """Executing the same batch plan twice on fresh copies gives the same bits."""
    mats, nbs, trees, variants = mixed_batch(12, seed=9, mhi=300)
    plan = bb.BatchPlan([A.shape for A in mats], nb=nbs, tree=trees, variant=variants, timing=True)
    outs = []
    for rep in range(2):
        buf, ptrs, ldas, offs = bb.pack_batch(mats)
        vt, ws = plan.alloc()
        plan.execute(ptrs, ldas, vt, ws)
        assert plan.poll_error(ws) == 0
        assert plan.last_kernel_ms() > 0.0
        outs.append(buf.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("prec", ["f64_upd_f32", "f64_upd_split32"])
def test_mixed_precision_batch(bb, prec):
    """Updates on FP32 matrix cores in a batch: every matrix within the FP32
    backward-error bound 50 n eps32 ||A|| of the oracle (the single-matrix
    precision tests use the same one), and bitwise equal to the same matrix
    reduced alone in that mode."""
    mats, nbs, trees, variants = mixed_batch(24, seed=17)
    print("mixed-precision batch", prec, len(mats), flush=True)
    plan, Bs = run_batch(bb, mats, nb=nbs, tree=trees, variant=variants, prec=prec)
    for i, (A, B) in enumerate(zip(mats, Bs)):
        n = A.shape[1]
        assert oracle.band_violation(B, nbs[i]) == 0.0, i
        Bo, _ = oracle.band_reduce(A, nbs[i])
        d = np.linalg.norm(oracle.sign_normalize(B, nbs[i]) - oracle.sign_normalize(Bo, nbs[i]))
        assert d <= 50 * n * 2.0 ** -24 * np.linalg.norm(A), (i, A.shape, d)
    for i in (0, 13, 23):
        Bsingle, _, _ = bb.band(torch.from_numpy(mats[i]), nbs[i], trees[i], variants[i], prec=prec)
        assert np.array_equal(Bsingle.cpu().numpy(), Bs[i]), i
