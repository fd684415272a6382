"""GPU tests of the C ABI's ownership contract (include/bidiag.h).

* The library allocates no device memory: the first execution of a new plan
  leaves the device's free memory unchanged (its graph goes into the caller's
  workspace with an asynchronous copy).
* The one-shot entry point is reentrant given distinct buffers: two host
  threads reducing the same shape at once, through one cached plan, on their
  own streams, give the bits of a single-threaded run.
* The adjoint's scheduler status is readable (bb_adjoint_poll_error).
"""
import ctypes
import threading

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


def test_first_execute_allocates_no_device_memory(bb):
    m, n, nb = 700, 450, 64
    A = workloads.gaussian(m, n, seed=77)
    # load the kernels' code object with another plan first
    bb.band(torch.from_numpy(A[:300, :200].copy()), nb, "greedy", "bidiag")
    plan = bb.Plan(m, n, nb, "greedy", "rbidiag")
    S = bb.to_colmajor(torch.from_numpy(A))
    vt, ws = plan.alloc(S.device)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    print("first execute of a new plan", m, n, nb, flush=True)
    plan.execute(S, m, vt, ws)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
    assert bb.poll_error(ws) == 0
    B = S.t().cpu().numpy()
    assert oracle.band_violation(B, nb) == 0.0
    Bo, _ = oracle.band_reduce(A, nb)
    d = np.linalg.norm(oracle.sign_normalize(B, nb) - oracle.sign_normalize(Bo, nb))
    assert d <= 50 * n * EPS * np.linalg.norm(A)


def _one_shot(bb, S, m, n, nb, vt, ws, stream):
    L = bb.lib()
    opts = bb.make_opts()
    return L.bidiag_band(ctypes.c_void_p(S.data_ptr()), m, n, m, nb, bb.TREES["greedy"],
                         bb.VARIANTS["rbidiag"], 0, ctypes.c_void_p(vt.data_ptr()), vt.numel(),
                         ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(opts),
                         ctypes.c_void_p(stream.cuda_stream))


def test_one_shot_from_two_threads(bb):
    m, n, nb = 900, 520, 64
    A = workloads.gaussian(m, n, seed=78)
    bb.cache_clear()
    vtb, wsb = bb.query(m, n, nb, "greedy", "rbidiag")
    S0 = bb.to_colmajor(torch.from_numpy(A))
    ref = S0.clone()
    vt = torch.empty(vtb, dtype=torch.uint8, device="cuda")
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    print("single-threaded one-shot", flush=True)
    assert _one_shot(bb, ref, m, n, nb, vt, ws, s) == 0
    s.synchronize()
    assert bb.poll_error(ws, s) == 0

    outs, rcs = [], [None, None]
    bufs = []
    for k in range(2):
        bufs.append((S0.clone(), torch.empty_like(vt), torch.empty_like(ws), torch.cuda.Stream()))
    torch.cuda.synchronize()

    def run(k):
        S, v, w, st = bufs[k]
        for it in range(4):
            with torch.cuda.stream(st):
                S.copy_(S0)
            rcs[k] = _one_shot(bb, S, m, n, nb, v, w, st)
            if rcs[k] != 0:
                return
            if k == 0 and it == 1:
                # evict the cached plan while the other thread may be using it
                bb.cache_clear()
        st.synchronize()

    print("two threads", flush=True)
    th = [threading.Thread(target=run, args=(k,)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    assert rcs == [0, 0], rcs
    for S, v, w, st in bufs:
        assert bb.poll_error(w, st) == 0
        assert torch.equal(S, ref)


def test_adjoint_status_is_reported(bb):
    m, n, nb = 600, 256, 64
    A = workloads.gaussian(m, n, seed=79)
    W = torch.as_tensor(workloads.band_weights(n, nb, 80)).cuda()
    plan = bb.Plan(m, n, nb, "greedy", "rbidiag")
    S = bb.to_colmajor(torch.from_numpy(A))
    vt, ws = plan.alloc(S.device)
    plan.execute(S, m, vt, ws)
    aws = torch.empty(plan.adjoint_workspace(), dtype=torch.uint8, device="cuda")
    # through the binding, which checks the status itself (this also loads
    # the adjoint's kernels)
    Ab2 = plan.adjoint(S, m, W, vt, ws=aws, check=True)
    Wcm = W.t().contiguous()
    Ab = torch.empty(n, m, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    print("adjoint", m, n, nb, flush=True)
    L = bb.lib()
    rc = L.bidiag_band_adjoint(plan._h, ctypes.c_void_p(S.data_ptr()), m, ctypes.c_void_p(Wcm.data_ptr()),
                               n, ctypes.c_void_p(vt.data_ptr()), vt.numel(),
                               ctypes.c_void_p(Ab.data_ptr()), m, ctypes.c_void_p(aws.data_ptr()),
                               aws.numel(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    assert plan.adjoint_poll_error(aws) == 0
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
    assert torch.isfinite(Ab).all()
    assert torch.equal(Ab2, Ab.t())
