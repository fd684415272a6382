"""GPU test of the persistent scheduler's watchdog, forced from the host.

A spin limit of zero clock ticks makes the first workgroup that finds its unit
not ready report BB_ETIMEOUT (3); every other workgroup stops at its next
wait, and units that were ready run to completion, so the launch ends
normally.  The error reaches the caller through bb_poll_error, and the same
shapes then reduce correctly with a normal limit: nothing of the failed launch
is left behind (the dependency counters and the error word are reset per
launch).
"""
import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
TINY = 1e-12     # seconds: zero ticks of the 100 MHz wall clock


@pytest.fixture(scope="module")
def bb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1611_06892_amd as m
    m.lib()
    return m


def close_to_oracle(A, B, nb):
    n = A.shape[1]
    assert oracle.band_violation(B, nb) == 0.0
    Bo, _ = oracle.band_reduce(A, nb)
    d = np.linalg.norm(oracle.sign_normalize(B, nb) - oracle.sign_normalize(Bo, nb))
    assert d <= 50 * n * EPS * np.linalg.norm(A), d


def test_watchdog_reports_timeout_and_the_next_launch_is_correct(bb):
    # 32 x 16 tiles: thousands of units, far more than the workgroups, so
    # some workgroup must wait for a dependency
    m, n, nb = 2048, 1024, 64
    A = workloads.gaussian(m, n, seed=4242)
    print("watchdog case", m, n, nb, flush=True)
    with pytest.raises(bb.BidiagError) as e:
        bb.band(torch.from_numpy(A), nb, "greedy", "rbidiag", watchdog_s=TINY)
    torch.cuda.synchronize()
    assert e.value.code == 3
    assert bb.strerror(3) == "device scheduler watchdog expired"
    print("recovery run", flush=True)
    B, _, _ = bb.band(torch.from_numpy(A), nb, "greedy", "rbidiag", watchdog_s=10.0)
    torch.cuda.synchronize()
    close_to_oracle(A, B.cpu().numpy(), nb)


def test_batch_watchdog_reports_timeout_and_recovers(bb):
    rng = np.random.default_rng(99)
    mats = []
    for _ in range(24):
        mm = int(rng.integers(300, 700))
        nn = int(rng.integers(200, mm + 1))
        mats.append(np.asfortranarray(rng.standard_normal((mm, nn))))
    shapes = [A.shape for A in mats]
    print("batch watchdog case", len(mats), flush=True)
    plan = bb.BatchPlan(shapes, nb=64, tree="greedy", variant="bidiag", watchdog_s=TINY)
    buf, ptrs, ldas, offs = bb.pack_batch(mats)
    vt, ws = plan.alloc()
    plan.execute(ptrs, ldas, vt, ws)
    assert plan.poll_error(ws) == 3
    torch.cuda.synchronize()
    print("batch recovery run", flush=True)
    plan = bb.BatchPlan(shapes, nb=64, tree="greedy", variant="bidiag", watchdog_s=20.0)
    buf, ptrs, ldas, offs = bb.pack_batch(mats)
    vt, ws = plan.alloc()
    plan.execute(ptrs, ldas, vt, ws)
    assert plan.poll_error(ws) == 0
    torch.cuda.synchronize()
    for i in (0, 11, 23):
        close_to_oracle(mats[i], bb.unpack(buf, offs, plan.shapes, i).cpu().numpy(), 64)
