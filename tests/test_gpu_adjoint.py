"""GPU tests of the band-form adjoint (bidiag_band_adjoint and the autograd
function): the gradient of L = sum(W * B) over the band against

  * the reference gradient of the oracle (autograd through block Golub-Kahan
    on the CPU, FP64, an independent algorithm), and
  * central finite differences of the GPU forward in random directions.
"""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1611_06892_amd as m
    m.lib()
    return m


def band_weights(n, nb, seed):
    rng = np.random.default_rng(seed)
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    return rng.standard_normal((n, n)) * ((j >= i) & (j <= i + nb))


def forward(bb, A, nb, tree, variant):
    m, n = A.shape
    plan = bb.Plan(m, n, nb, tree, variant, watchdog_s=20.0)
    S = torch.as_tensor(A).cuda().t().contiguous()
    vt, ws = plan.alloc()
    plan.execute(S, m, vt, ws)
    assert bb.poll_error(ws) == 0
    return plan, S, vt


CASES = [
    (160, 96, 32, "greedy", "bidiag"),
    (200, 130, 32, "flatts", "rbidiag"),     # ragged
    (256, 256, 64, "auto", "bidiag"),
    (640, 256, 128, "greedy", "rbidiag"),
    (300, 100, 64, "flattt", "bidiag"),      # ragged, q = 2
    (150, 40, 64, "greedy", "bidiag"),       # n < nb: the QR adjoint
]


@pytest.mark.parametrize("m,n,nb,tree,variant", CASES)
def test_adjoint_matches_reference_gradient(bb, m, n, nb, tree, variant):
    from oracle import adjoint as ref
    print("case", m, n, nb, tree, variant, flush=True)
    A = workloads.gaussian(m, n, seed=500 + m + n + nb)
    W = band_weights(n, nb, seed=n)
    plan, S, vt = forward(bb, A, nb, tree, variant)
    Ab = plan.adjoint(S, m, torch.as_tensor(W), vt)
    torch.cuda.synchronize()
    Ag = Ab.cpu().numpy()
    B = S.t().cpu().numpy()
    _, Aref = ref.band_loss_gradient(A, W, nb, B)
    rel = np.linalg.norm(Ag - Aref) / np.linalg.norm(Aref)
    print("relative difference to the reference gradient", rel, flush=True)
    assert rel <= 1e-9


@pytest.mark.parametrize("m,n,nb,tree,variant", CASES[:4])
def test_adjoint_finite_differences(bb, m, n, nb, tree, variant):
    print("case", m, n, nb, tree, variant, flush=True)
    A = workloads.gaussian(m, n, seed=900 + m + n)
    W = band_weights(n, nb, seed=n + 1)
    plan, S, vt = forward(bb, A, nb, tree, variant)
    Ag = plan.adjoint(S, m, torch.as_tensor(W), vt).cpu().numpy()
    Wd = torch.as_tensor(W).cuda()

    def L(M):
        _, Sm, _ = forward(bb, M, nb, tree, variant)
        return float(torch.sum(Wd * Sm.t()[:n]))

    rng = np.random.default_rng(7)
    h = 1e-6 * np.linalg.norm(A)
    for _ in range(8):
        E = rng.standard_normal((m, n))
        E /= np.linalg.norm(E)
        fd = (L(A + h * E) - L(A - h * E)) / (2 * h)
        an = float(np.sum(Ag * E))
        assert abs(fd - an) <= 1e-6 * max(1.0, np.linalg.norm(Ag)), (fd, an)


def block_condition(B, n, nb):
    """Largest 2-norm condition number of the diagonal and super-diagonal
    nb-blocks of the band B (the blocks the reverse sweep solves with)."""
    kappa = 1.0
    for k0 in range(0, n, nb):
        k1 = min(k0 + nb, n)
        kappa = max(kappa, np.linalg.cond(B[k0:k1, k0:k1]))
        if k1 < n:
            kappa = max(kappa, np.linalg.cond(B[k0:k1, k1:min(k1 + nb, n)]))
    return kappa


@pytest.mark.parametrize("prec", ["f64_upd_f32", "f64_upd_split32"])
@pytest.mark.parametrize("m,n,nb,tree,variant", [CASES[0], CASES[3]])
def test_adjoint_of_mixed_precision_forward(bb, prec, m, n, nb, tree, variant):
    """Forward with FP32 (or split-FP32) updates, adjoint in FP64 from its
    records.  The mixed forward reduces A + dA exactly with ||dA|| within
    50 n eps32 ||A|| (the bound of the mixed-precision band tests), and the
    reverse sweep solves with the diagonal and super-diagonal blocks of B, so
    the gradient of the reference moves by at most that relative amount times
    the blocks' largest condition number."""
    from oracle import adjoint as ref
    print("case", prec, m, n, nb, tree, variant, flush=True)
    A = workloads.gaussian(m, n, seed=700 + m + n + nb)
    W = band_weights(n, nb, seed=n + 2)
    plan = bb.Plan(m, n, nb, tree, variant, prec=prec, watchdog_s=20.0)
    S = torch.as_tensor(A).cuda().t().contiguous()
    vt, ws = plan.alloc()
    plan.execute(S, m, vt, ws)
    assert bb.poll_error(ws) == 0
    Ag = plan.adjoint(S, m, torch.as_tensor(W), vt).cpu().numpy()
    B = S.t().cpu().numpy()
    _, Aref = ref.band_loss_gradient(A, W, nb, B)
    rel = np.linalg.norm(Ag - Aref) / np.linalg.norm(Aref)
    kappa = block_condition(B, n, nb)
    print("relative difference", rel, "block condition", kappa, flush=True)
    assert rel <= 50 * n * 2.0 ** -24 * kappa


def test_autograd_function(bb):
    m, n, nb = 300, 192, 64
    A = torch.as_tensor(workloads.gaussian(m, n, seed=3)).cuda().requires_grad_(True)
    Wt = torch.as_tensor(band_weights(n, nb, seed=4)).cuda()
    B = bb.band_autograd(A, nb, "greedy", "rbidiag")
    loss = torch.sum(Wt * B[:n])
    (g,) = torch.autograd.grad(loss, A)
    plan, S, vt = forward(bb, A.detach().cpu().numpy(), nb, "greedy", "rbidiag")
    direct = plan.adjoint(S, m, Wt, vt)
    assert torch.allclose(g, direct, rtol=0, atol=1e-12 * float(torch.linalg.norm(direct)))


def test_adjoint_full_size(bb):
    """8192 x 1024 N(0,1) (seed 6), band weights N(0,1) (seed 7), nb = 128,
    R-BiDiag: finite differences of the GPU forward in 4 random directions."""
    cfg = workloads.CONFIGS["adjoint"]
    m, n, nb = cfg["m"], cfg["n"], cfg["nb"]
    print("case adjoint full size", flush=True)
    A = workloads.gaussian(m, n, cfg["seed"])
    W = workloads.band_weights(n, nb, cfg["wseed"])
    plan, S, vt = forward(bb, A, nb, "greedy", "rbidiag")
    Ag = plan.adjoint(S, m, torch.as_tensor(W), vt).cpu().numpy()
    Wd = torch.as_tensor(W).cuda()

    def L(M):
        _, Sm, _ = forward(bb, M, nb, "greedy", "rbidiag")
        return float(torch.sum(Wd * Sm.t()[:n]))

    rng = np.random.default_rng(8)
    h = 1e-6 * np.linalg.norm(A)
    nAg = np.linalg.norm(Ag)
    for _ in range(4):
        E = rng.standard_normal((m, n))
        E /= np.linalg.norm(E)
        fd = (L(A + h * E) - L(A - h * E)) / (2 * h)
        an = float(np.sum(Ag * E))
        print("fd", fd, "adjoint", an, "|grad|", nAg, flush=True)
        assert abs(fd - an) <= 1e-5 * nAg


def test_band_does_not_modify_its_input(bb):
    """Regression: a column-major FP64 CUDA input (Fortran strides) must be
    copied, not reduced in place."""
    A0 = workloads.gaussian(300, 192, seed=3)
    A = torch.as_tensor(A0).cuda()
    assert A.stride() == (1, 300)
    B, _, _ = bb.band(A, 64, "greedy", "rbidiag")
    torch.cuda.synchronize()
    assert np.array_equal(A.cpu().numpy(), A0)
    Ag = A.clone().requires_grad_(True)
    bb.band_autograd(Ag, 64, "greedy", "rbidiag")
    assert np.array_equal(Ag.detach().cpu().numpy(), A0)
