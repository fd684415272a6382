"""GPU test of the persistent scheduler through its trace (bb_plan_trace).

Every work unit of the ticket order runs exactly once; its ticket is taken
before it starts and it starts before it ends; and no unit starts before every
unit of every predecessor task has ended, i.e. the dependency counters and the
completion signal (given only after a unit's outputs are complete, possibly
while the workgroup already loads its next unit) order the graph.  The band
result is checked against the oracle as well.
"""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1611_06892_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("m,n,nb,tree,variant", [
    (1024, 512, 64, "greedy", "rbidiag"),
    (700, 700, 32, "auto", "bidiag"),
    (2048, 384, 128, "flatts", "bidiag"),
])
def test_trace_respects_the_task_graph(bb, m, n, nb, tree, variant):
    print("case", m, n, nb, tree, variant, flush=True)
    rng = np.random.default_rng(m + n + nb)
    A = np.asfortranarray(rng.standard_normal((m, n)))
    S = bb.to_colmajor(torch.from_numpy(A).cuda())
    plan = bb.Plan(m, n, nb, tree, variant, trace=True, watchdog_s=10.0)
    vt, ws = plan.alloc()
    plan.execute(S, m, vt, ws)
    torch.cuda.synchronize()
    assert bb.poll_error(ws) == 0
    tr = plan.trace(ws)
    tasks, off, idx = plan.export()
    nt = len(off) - 1

    # Every task runs, each of its units (parts 0, 1, ...) exactly once, and a
    # panel task is one unit.
    parts = {}
    for t, p in zip(tr["task"], tr["part"]):
        parts.setdefault(int(t), []).append(int(p))
    assert sorted(parts) == list(range(nt))
    for t, ps in parts.items():
        assert sorted(ps) == list(range(len(ps)))
        if tasks[t, 0] <= 2:
            assert ps == [0]

    # Times in order per unit; workgroups within the grid.
    assert np.all(tr["wait"] <= tr["start"]) and np.all(tr["start"] <= tr["end"])
    assert tr["workgroup"].min() >= 0 and tr["workgroup"].max() < 4096

    # No unit starts before all units of its predecessor tasks have ended.
    first = np.full(nt, np.inf)
    last = np.zeros(nt)
    np.minimum.at(first, tr["task"], tr["start"])
    np.maximum.at(last, tr["task"], tr["end"])
    for t in range(nt):
        preds = idx[off[t]:off[t + 1]]
        if len(preds):
            assert first[t] >= last[preds].max(), "task %d started before a predecessor ended" % t

    # And the result is the oracle's band form (up to the signs of B's
    # rows and columns).
    Bg = S.t().cpu().numpy()
    assert oracle.band_violation(Bg, nb) == 0.0
    Bo, _ = oracle.band_reduce(A, nb)
    d = np.linalg.norm(oracle.sign_normalize(Bg, nb) - oracle.sign_normalize(Bo, nb))
    assert d <= 50.0 * n * np.finfo(np.float64).eps * np.linalg.norm(A)
