"""Python binding of libbidiag: tiled band bidiagonalization on MI355X (gfx950).

Thin ctypes layer over the C ABI in ``include/bidiag.h``: it marshals
arguments and uses PyTorch only for device memory and the current HIP stream.
Every step of the reduction runs in the library's HIP kernels; if the library
is missing this module raises instead of computing anything itself.

Band form (Sections 3.4 and 3.5 of the paper): B = Q^T A P with B(i,j) = 0
unless 0 <= j - i <= nb, reached by BiDiag or R-BiDiag with the FlatTS,
FlatTT, Greedy or Auto reduction trees.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbidiag.so")

TREES = {"flatts": 0, "flattt": 1, "greedy": 2, "auto": 3}
VARIANTS = {"bidiag": 0, "rbidiag": 1, "qronly": 2, "threestep": 3}
PRECS = {"f64": 0, "f64_upd_f32": 2, "f64_upd_split32": 3}
SCHEDS = {"persistent": 0, "levels": 1}
KINDS = ["GEQRT", "TSQRT", "TTQRT", "UNMQR", "TSMQR", "TTMQR"]
FLAG_TIMING = 1
FLAG_TRACE = 2


class BidiagError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__("%s failed: %s (code %d)" % (where, strerror(code), code))


class _Opts(ctypes.Structure):
    _fields_ = [("workgroups", ctypes.c_int), ("gamma", ctypes.c_double),
                ("auto_a", ctypes.c_int), ("sched", ctypes.c_int),
                ("watchdog_s", ctypes.c_double), ("flags", ctypes.c_int),
                ("switch_step", ctypes.c_int), ("delta", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("q", ctypes.c_int32), ("nb", ctypes.c_int32),
                ("ntasks", ctypes.c_int64), ("nunits", ctypes.c_int64),
                ("nslots", ctypes.c_int64), ("nlevels", ctypes.c_int64),
                ("count_by_kind", ctypes.c_int64 * 6), ("critical_path", ctypes.c_double),
                ("total_weight", ctypes.c_double)]


_lib = None

# Every symbol include/bidiag.h declares.
EXPORTS = ["bb_plan_create", "bb_plan_destroy", "bb_plan_workspace", "bb_plan_get_stats",
           "bb_plan_export", "bb_execute", "bidiag_band", "bb_query", "bb_poll_error",
           "bb_plan_last_kernel_ms", "bb_critical_path", "bb_strerror", "bb_graph_check",
           "bb_plan_auto_domains", "bb_apply_q", "bb_apply_p", "bb_apply_workspace",
           "bb_tuned_config", "bb_batch_create", "bb_batch_destroy", "bb_batch_workspace",
           "bb_batch_info", "bb_batch_execute", "bb_batch_last_kernel_ms", "bb_batch_poll_error",
           "bb_query_batched", "bidiag_band_batched", "bidiag_band_adjoint",
           "bb_adjoint_workspace", "bb_adjoint_poll_error", "bb_plan_trace", "bb_cache_clear",
           "bb_execute_noalloc", "bb_choose", "bb_bnd2bd_workspace", "bb_bnd2bd", "bb_bnd2bd_group", "bb_bd2val",
           "bb_ge2val_workspace", "bb_ge2val"]


def lib():
    """Load libbidiag.so (built by ``python -m paper_1611_06892_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libbidiag.so is not built (%s); run python -m "
                          "paper_1611_06892_amd.build" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    P = ctypes.c_void_p
    L.bb_plan_create.argtypes = [ctypes.POINTER(P), i64, i64, i32, i32, i32, i32,
                                 ctypes.POINTER(_Opts)]
    L.bb_plan_create.restype = i32
    L.bb_plan_destroy.argtypes = [P]
    L.bb_plan_destroy.restype = None
    L.bb_plan_workspace.argtypes = [P, ctypes.POINTER(ctypes.c_size_t),
                                    ctypes.POINTER(ctypes.c_size_t)]
    L.bb_plan_workspace.restype = i32
    L.bb_plan_get_stats.argtypes = [P, ctypes.POINTER(_Stats)]
    L.bb_plan_get_stats.restype = i32
    L.bb_plan_export.argtypes = [P, vp, vp, vp, ctypes.POINTER(i64)]
    L.bb_plan_export.restype = i32
    L.bb_execute.argtypes = [P, vp, i64, vp, ctypes.c_size_t, vp, ctypes.c_size_t, vp]
    L.bb_execute.restype = i32
    L.bidiag_band.argtypes = [vp, i64, i64, i64, i32, i32, i32, i32, vp, ctypes.c_size_t, vp,
                              ctypes.c_size_t, ctypes.POINTER(_Opts), vp]
    L.bidiag_band.restype = i32
    L.bb_query.argtypes = [i64, i64, i32, i32, i32, i32, ctypes.POINTER(_Opts),
                           ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
    L.bb_query.restype = i32
    L.bb_poll_error.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int)]
    L.bb_poll_error.restype = i32
    L.bb_plan_last_kernel_ms.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
    L.bb_plan_last_kernel_ms.restype = i32
    L.bb_critical_path.argtypes = [i32, i32, i32, i32, i32, i32, ctypes.c_double]
    L.bb_critical_path.restype = ctypes.c_double
    L.bb_graph_check.argtypes = [i32, i32, i64, vp, vp, vp]
    L.bb_graph_check.restype = i32
    L.bb_plan_auto_domains.argtypes = [P, vp, ctypes.POINTER(i64)]
    L.bb_plan_auto_domains.restype = i32
    for name in ("bb_apply_q", "bb_apply_p"):
        f = getattr(L, name)
        f.argtypes = [P, i32, vp, ctypes.c_size_t, vp, i64, i64, vp, ctypes.c_size_t, vp]
        f.restype = i32
    L.bb_apply_workspace.argtypes = [P, i32, i32, i64, ctypes.POINTER(ctypes.c_size_t)]
    L.bb_apply_workspace.restype = i32
    ip, lp = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64)
    szp = ctypes.POINTER(ctypes.c_size_t)
    L.bb_tuned_config.argtypes = [i64, i64, i32, ip, ip, ip]
    L.bb_tuned_config.restype = i32
    L.bb_batch_create.argtypes = [ctypes.POINTER(P), i64, vp, vp, vp, vp, vp, i32,
                                  ctypes.POINTER(_Opts)]
    L.bb_batch_create.restype = i32
    L.bb_batch_destroy.argtypes = [P]
    L.bb_batch_destroy.restype = None
    L.bb_batch_workspace.argtypes = [P, szp, szp]
    L.bb_batch_workspace.restype = i32
    L.bb_batch_info.argtypes = [P, i64, ip, ip, ip, lp, lp]
    L.bb_batch_info.restype = i32
    L.bb_batch_execute.argtypes = [P, vp, vp, vp, ctypes.c_size_t, vp, ctypes.c_size_t, vp]
    L.bb_batch_execute.restype = i32
    L.bb_batch_last_kernel_ms.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
    L.bb_batch_last_kernel_ms.restype = i32
    L.bb_batch_poll_error.argtypes = [P, vp, vp, ip]
    L.bb_batch_poll_error.restype = i32
    L.bb_query_batched.argtypes = [i64, vp, vp, vp, vp, vp, i32, ctypes.POINTER(_Opts), szp, szp]
    L.bb_query_batched.restype = i32
    L.bidiag_band_batched.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, i32, vp, ctypes.c_size_t,
                                      vp, ctypes.c_size_t, ctypes.POINTER(_Opts), vp]
    L.bidiag_band_batched.restype = i32
    L.bidiag_band_adjoint.argtypes = [P, vp, i64, vp, i64, vp, ctypes.c_size_t, vp, i64, vp,
                                      ctypes.c_size_t, vp]
    L.bidiag_band_adjoint.restype = i32
    L.bb_adjoint_workspace.argtypes = [P, szp]
    L.bb_adjoint_workspace.restype = i32
    L.bb_adjoint_poll_error.argtypes = [P, vp, vp, ip]
    L.bb_adjoint_poll_error.restype = i32
    L.bb_choose.argtypes = [i64, i64, i32, ctypes.POINTER(_Opts), ip, ip, ctypes.POINTER(ctypes.c_double)]
    L.bb_choose.restype = i32
    L.bb_execute_noalloc.argtypes = [P, vp, i64, vp, ctypes.c_size_t, vp]
    L.bb_execute_noalloc.restype = i32
    L.bb_bnd2bd_workspace.argtypes = [i64, i32, szp]
    L.bb_bnd2bd_workspace.restype = i32
    L.bb_bnd2bd.argtypes = [vp, i64, i64, i32, vp, vp, vp, ctypes.c_size_t, ctypes.c_double, vp]
    L.bb_bnd2bd.restype = i32
    L.bb_bnd2bd_group.argtypes = [vp, i64, i64, i32, vp, vp, vp, ctypes.c_size_t, ctypes.c_double, i32, vp]
    L.bb_bnd2bd_group.restype = i32
    L.bb_bd2val.argtypes = [vp, vp, i64, vp, vp]
    L.bb_bd2val.restype = i32
    L.bb_ge2val_workspace.argtypes = [i64, i64, i32, i32, i32, i32, ctypes.POINTER(_Opts),
                                      ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
    L.bb_ge2val_workspace.restype = i32
    L.bb_ge2val.argtypes = [vp, i64, i64, i64, i32, i32, i32, i32, vp, vp, ctypes.c_size_t, vp, ctypes.c_size_t,
                            ctypes.POINTER(_Opts), vp]
    L.bb_ge2val.restype = i32
    L.bb_cache_clear.argtypes = []
    L.bb_cache_clear.restype = None
    L.bb_plan_trace.argtypes = [P, szp, lp, ctypes.POINTER(ctypes.c_double), vp]
    L.bb_plan_trace.restype = i32
    L.bb_strerror.argtypes = [i32]
    L.bb_strerror.restype = ctypes.c_char_p
    _lib = L
    return L


def query(m, n, nb, tree="auto", variant="bidiag", prec="f64", **opts):
    """(vt_bytes, ws_bytes) for bidiag_band with these arguments (bb_query)."""
    o = make_opts(**opts)
    vt, ws = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().bb_query(int(m), int(n), int(nb), TREES[tree], VARIANTS[variant], PRECS[prec],
                          ctypes.byref(o), ctypes.byref(vt), ctypes.byref(ws)), "bb_query")
    return vt.value, ws.value


def choose(m, n, nb, **opts):
    """(tree, variant, estimate): the shortest estimated schedule among BiDiag,
    R-BiDiag and the three-step reduction with the Greedy and Auto trees."""
    o = make_opts(**opts)
    tr, var, est = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    _check(lib().bb_choose(int(m), int(n), int(nb), ctypes.byref(o), ctypes.byref(tr), ctypes.byref(var),
                           ctypes.byref(est)), "bb_choose")
    return TREE_NAMES[tr.value], VARIANT_NAMES[var.value], est.value


def cache_clear():
    """Drop the plans the one-shot entry points cache."""
    lib().bb_cache_clear()


def strerror(code: int) -> str:
    return lib().bb_strerror(int(code)).decode()


def _check(rc: int, where: str):
    if rc != 0:
        raise BidiagError(rc, where)


def make_opts(workgroups=0, gamma=0.0, auto_a=0, sched="persistent", watchdog_s=0.0,
              timing=False, trace=False, switch_step=0, delta=0.0) -> _Opts:
    return _Opts(int(workgroups), float(gamma), int(auto_a), SCHEDS[sched], float(watchdog_s),
                 (FLAG_TIMING if timing else 0) | (FLAG_TRACE if trace else 0),
                 int(switch_step), float(delta))


def critical_path(p: int, q: int, tree="greedy", variant="bidiag", auto_a=0, workgroups=256,
                  gamma=2.0) -> float:
    """Critical path (Section 4) in units of nb^3/3 with Table 1 weights."""
    return lib().bb_critical_path(p, q, TREES[tree], VARIANTS[variant], auto_a, workgroups, gamma)


def graph_check(p, q, tasks, pred_off, pred_idx) -> int:
    """Static race check of an exported task graph (BB_OK = 0 or BB_EDAG)."""
    tasks = np.ascontiguousarray(tasks, dtype=np.int32)
    pred_off = np.ascontiguousarray(pred_off, dtype=np.int32)
    pred_idx = np.ascontiguousarray(pred_idx, dtype=np.int32)
    if pred_idx.size == 0:
        pred_idx = np.zeros(1, dtype=np.int32)
    return lib().bb_graph_check(int(p), int(q), int(tasks.shape[0]), tasks.ctypes.data,
                                pred_off.ctypes.data, pred_idx.ctypes.data)


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """Task graph and schedule of one (m, n, nb, tree, variant) reduction."""

    def __init__(self, m, n, nb, tree="auto", variant="bidiag", prec="f64", **opts):
        self.m, self.n, self.nb = int(m), int(n), int(nb)
        self.tree, self.variant, self.prec = tree, variant, prec
        self._opts = make_opts(**opts)
        h = ctypes.c_void_p()
        _check(lib().bb_plan_create(ctypes.byref(h), self.m, self.n, self.nb, TREES[tree],
                                    VARIANTS[variant], PRECS[prec], ctypes.byref(self._opts)),
               "bb_plan_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.bb_plan_destroy(h)
            self._h = None

    def workspace(self):
        vt, ws = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().bb_plan_workspace(self._h, ctypes.byref(vt), ctypes.byref(ws)),
               "bb_plan_workspace")
        return vt.value, ws.value

    def stats(self) -> dict:
        s = _Stats()
        _check(lib().bb_plan_get_stats(self._h, ctypes.byref(s)), "bb_plan_get_stats")
        return {"p": s.p, "q": s.q, "nb": s.nb, "ntasks": s.ntasks, "nunits": s.nunits,
                "nslots": s.nslots, "nlevels": s.nlevels,
                "count_by_kind": dict(zip(KINDS, list(s.count_by_kind))),
                "critical_path": s.critical_path, "total_weight": s.total_weight}

    def export(self):
        """(tasks[ntasks, 8], pred_off[ntasks+1], pred_idx[npred]) as int32 arrays."""
        npred = ctypes.c_int64()
        _check(lib().bb_plan_export(self._h, None, None, None, ctypes.byref(npred)),
               "bb_plan_export")
        nt = self.stats()["ntasks"]
        tasks = np.zeros((nt, 8), dtype=np.int32)
        off = np.zeros(nt + 1, dtype=np.int32)
        idx = np.zeros(max(1, npred.value), dtype=np.int32)
        _check(lib().bb_plan_export(self._h, tasks.ctypes.data, off.ctypes.data, idx.ctypes.data,
                                    ctypes.byref(npred)), "bb_plan_export")
        return tasks, off, idx[:npred.value]

    def auto_domains(self):
        """Auto's FlatTS domain size per QR/LQ step (0 for other trees)."""
        ns = ctypes.c_int64()
        _check(lib().bb_plan_auto_domains(self._h, None, ctypes.byref(ns)), "bb_plan_auto_domains")
        out = np.zeros(max(1, ns.value), dtype=np.int32)
        _check(lib().bb_plan_auto_domains(self._h, out.ctypes.data, ctypes.byref(ns)),
               "bb_plan_auto_domains")
        return out[:ns.value]

    def alloc(self, device=None):
        """Allocate (vt, ws) byte buffers of the sizes this plan needs."""
        import torch
        vt_b, ws_b = self.workspace()
        dev = device if device is not None else torch.device("cuda")
        vt = torch.empty(max(vt_b, 8), dtype=torch.uint8, device=dev)
        ws = torch.empty(max(ws_b, 8), dtype=torch.uint8, device=dev)
        return vt, ws

    def execute(self, Acm, lda, vt, ws, stream=None):
        """Reduce the column-major matrix at Acm (a CUDA tensor whose storage is
        m x n column-major with leading dimension lda) in place."""
        _check(lib().bb_execute(self._h, ctypes.c_void_p(Acm.data_ptr()), int(lda),
                                ctypes.c_void_p(vt.data_ptr()), vt.numel() * vt.element_size(),
                                ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                _stream_handle(stream)), "bb_execute")

    def execute_noalloc(self, Acm, lda, vt, stream=None):
        """bb_execute with the library's own per-device workspace (no device
        allocation; overlapping calls on one device race)."""
        _check(lib().bb_execute_noalloc(self._h, ctypes.c_void_p(Acm.data_ptr()), int(lda),
                                        ctypes.c_void_p(vt.data_ptr()),
                                        vt.numel() * vt.element_size(), _stream_handle(stream)),
               "bb_execute_noalloc")

    def apply_workspace(self, side, transpose, ncols) -> int:
        ws = ctypes.c_size_t()
        _check(lib().bb_apply_workspace(self._h, int(side), int(transpose), int(ncols),
                                        ctypes.byref(ws)), "bb_apply_workspace")
        return ws.value

    def _apply(self, side, Ccm, ldc, ncols, vt, transpose, ws, stream):
        import torch
        if ws is None:
            ws = torch.empty(max(self.apply_workspace(side, transpose, ncols), 8),
                             dtype=torch.uint8, device=Ccm.device)
        fn = lib().bb_apply_q if side == 0 else lib().bb_apply_p
        _check(fn(self._h, int(bool(transpose)), ctypes.c_void_p(vt.data_ptr()),
                  vt.numel() * vt.element_size(), ctypes.c_void_p(Ccm.data_ptr()), int(ldc),
                  int(ncols), ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                  _stream_handle(stream)), "bb_apply_q" if side == 0 else "bb_apply_p")
        return ws

    def apply_q(self, Ccm, ldc, ncols, vt, transpose=False, ws=None, stream=None):
        """C <- Q C (or Q^T C) in place; C is m x ncols column-major at Ccm."""
        return self._apply(0, Ccm, ldc, ncols, vt, transpose, ws, stream)

    def apply_p(self, Ccm, ldc, ncols, vt, transpose=False, ws=None, stream=None):
        """C <- P C (or P^T C) in place; C is n x ncols column-major at Ccm."""
        return self._apply(1, Ccm, ldc, ncols, vt, transpose, ws, stream)

    def last_kernel_ms(self) -> float:
        ms = ctypes.c_double()
        _check(lib().bb_plan_last_kernel_ms(self._h, ctypes.byref(ms)), "bb_plan_last_kernel_ms")
        return ms.value

    def trace(self, ws):
        """Per-unit records of the last persistent execution (trace=True plans):
        a dict of numpy arrays task, part, kind, wait, start, end (seconds from
        the first start) and workgroup."""
        off, nu, hz = ctypes.c_size_t(), ctypes.c_int64(), ctypes.c_double()
        _check(lib().bb_plan_trace(self._h, ctypes.byref(off), ctypes.byref(nu), ctypes.byref(hz),
                                   None), "bb_plan_trace")
        units = np.zeros(2 * max(nu.value, 1), dtype=np.int32)
        _check(lib().bb_plan_trace(self._h, None, None, None, units.ctypes.data), "bb_plan_trace")
        raw = ws[off.value: off.value + 32 * nu.value].view(-1).cpu().numpy().view(np.int64)
        raw = raw.reshape(nu.value, 4)
        tasks, _, _ = self.export()
        t0 = raw[:, 1].min() if nu.value else 0
        task = units[0:2 * nu.value:2]
        return {"task": task, "part": units[1:2 * nu.value:2], "kind": tasks[task, 0],
                "wait": (raw[:, 0] - t0) / hz.value, "start": (raw[:, 1] - t0) / hz.value,
                "end": (raw[:, 2] - t0) / hz.value, "workgroup": raw[:, 3]}

    def adjoint_workspace(self) -> int:
        ws = ctypes.c_size_t()
        _check(lib().bb_adjoint_workspace(self._h, ctypes.byref(ws)), "bb_adjoint_workspace")
        return ws.value

    def adjoint_poll_error(self, ws, stream=None) -> int:
        """Scheduler status of the last adjoint on ws (synchronizes the stream)."""
        st = ctypes.c_int()
        _check(lib().bb_adjoint_poll_error(self._h, ctypes.c_void_p(ws.data_ptr()),
                                           _stream_handle(stream), ctypes.byref(st)),
               "bb_adjoint_poll_error")
        return st.value

    def adjoint(self, Bcm, ldb, W, vt, ws=None, stream=None, check=False):
        """Gradient of sum(W * B) over the band with respect to the reduced
        matrix: Bcm is the column-major storage of the reduction's output B
        (leading dimension ldb), W an n x n tensor (only its band entries are
        used).  Returns the m x n gradient (a CUDA tensor view).  check=True
        waits for the result and raises BidiagError on a scheduler error."""
        import torch
        Wcm = W.to(device=Bcm.device, dtype=torch.float64).t().contiguous()
        Ab = torch.empty(self.n, self.m, dtype=torch.float64, device=Bcm.device)
        if ws is None:
            ws = torch.empty(max(self.adjoint_workspace(), 8), dtype=torch.uint8, device=Bcm.device)
        _check(lib().bidiag_band_adjoint(self._h, ctypes.c_void_p(Bcm.data_ptr()), int(ldb),
                                         ctypes.c_void_p(Wcm.data_ptr()), self.n,
                                         ctypes.c_void_p(vt.data_ptr()), vt.numel(),
                                         ctypes.c_void_p(Ab.data_ptr()), self.m,
                                         ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                         _stream_handle(stream)), "bidiag_band_adjoint")
        if check:
            st = self.adjoint_poll_error(ws, stream)
            if st != 0:
                raise BidiagError(st, "device scheduler (adjoint)")
        return Ab.t()


def poll_error(ws, stream=None) -> int:
    """Scheduler status of the last execution on workspace ws (synchronizes the
    stream); ws=None: of the last bb_execute_noalloc on the current device."""
    st = ctypes.c_int()
    wp = ctypes.c_void_p(ws.data_ptr()) if ws is not None else None
    _check(lib().bb_poll_error(wp, _stream_handle(stream), ctypes.byref(st)), "bb_poll_error")
    return st.value


def to_colmajor(A):
    """Column-major device copy of a 2-D tensor: returns the (n, m) row-major
    storage tensor S with S[j, i] = A[i, j] (so S.t() is A)."""
    import torch
    # always a copy: for a column-major FP64 CUDA input, .t().contiguous()
    # would return a view of the caller's storage, which the reduction
    # overwrites in place
    return A.to(device="cuda", dtype=torch.float64).t().clone(memory_format=torch.contiguous_format)


def band(A, nb, tree="auto", variant="bidiag", plan=None, check=True, **opts):
    """Band-bidiagonalize A (m x n, m >= n).  Returns (B, vt, plan) where B is
    an m x n CUDA tensor view holding the band form and vt the reflector
    records.  A is not modified."""
    m, n = A.shape
    S = to_colmajor(A)
    if plan is None:
        plan = Plan(m, n, nb, tree, variant, **opts)
    vt, ws = plan.alloc(S.device)
    plan.execute(S, m, vt, ws)
    if check:
        st = poll_error(ws)
        if st != 0:
            raise BidiagError(st, "device scheduler")
    return S.t(), vt, plan


def bnd2bd_workspace(n, nb) -> int:
    """Workspace bytes of bnd2bd for an n x n band of bandwidth nb."""
    b = ctypes.c_size_t()
    _check(lib().bb_bnd2bd_workspace(int(n), int(nb), ctypes.byref(b)), "bb_bnd2bd_workspace")
    return b.value


def bnd2bd(S, ldb, n, nb, ws=None, watchdog_s=0.0, stream=None, check=True, group=0):
    """Band to bidiagonal (bb_bnd2bd, or bb_bnd2bd_group with group > 0: the
    workgroups per sweep for nb > 64).  S: CUDA FP64 storage of a column-major
    matrix whose leading n x n part holds the upper band of bandwidth nb
    (leading dimension ldb), e.g. the storage tensor a Plan reduced.
    Returns (d, e) as CUDA tensors; S is not modified."""
    import torch
    dev = S.device
    if ws is None:
        ws = torch.empty(max(bnd2bd_workspace(n, nb), 8), dtype=torch.uint8, device=dev)
    d = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    e = torch.empty(max(n - 1, 1), dtype=torch.float64, device=dev)
    _check(lib().bb_bnd2bd_group(ctypes.c_void_p(S.data_ptr()), int(ldb), int(n), int(nb),
                                 ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(e.data_ptr()),
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(), float(watchdog_s), int(group),
                                 _stream_handle(stream)), "bb_bnd2bd_group")
    if check:
        st = poll_error(ws, stream)
        if st != 0:
            raise BidiagError(st, "bnd2bd sweep pipeline")
    return d[:n], e[:max(n - 1, 0)]


def bd2val(d, e, stream=None):
    """Singular values of the upper bidiagonal (d, e) in decreasing order
    (bb_bd2val), as a CUDA tensor."""
    import torch
    n = d.numel()
    d = d.to(dtype=torch.float64).contiguous()
    e = e.to(device=d.device, dtype=torch.float64).contiguous()
    sigma = torch.empty(max(n, 1), dtype=torch.float64, device=d.device)
    _check(lib().bb_bd2val(ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(e.data_ptr()), int(n),
                           ctypes.c_void_p(sigma.data_ptr()), _stream_handle(stream)), "bb_bd2val")
    return sigma[:n]


def ge2val(A, nb, tree="auto", variant="bidiag", **opts):
    """Singular values of A by GE2BND + BND2BD + BD2VAL, all on the GPU
    (decreasing order, a CUDA tensor).  A is not modified."""
    m, n = A.shape
    if m < n:
        return ge2val(A.t(), nb, tree, variant, **opts)
    B, vt, plan = band(A, nb, tree, variant, **opts)
    S = B.t()                      # the column-major storage, leading dimension m
    d, e = bnd2bd(S, m, n, nb)
    return bd2val(d, e)


def ge2val_oneshot(A, nb, tree="auto", variant="bidiag", prec="f64", stream=None, check=True, **opts):
    """Singular values of A through the C one-shot bb_ge2val (GE2BND, BND2BD
    and BD2VAL in stream order, one workspace), in decreasing order, as a
    CUDA tensor.  A is not modified (the reduction runs on a copy)."""
    import torch
    m, n = A.shape
    S = to_colmajor(A)
    o = make_opts(**opts)
    vtb, wsb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().bb_ge2val_workspace(int(m), int(n), int(nb), TREES[tree], VARIANTS[variant], PRECS[prec],
                                     ctypes.byref(o), ctypes.byref(vtb), ctypes.byref(wsb)), "bb_ge2val_workspace")
    vt = torch.empty(max(vtb.value, 8), dtype=torch.uint8, device=S.device)
    ws = torch.empty(max(wsb.value, 8), dtype=torch.uint8, device=S.device)
    k = min(m, n)
    sigma = torch.empty(max(k, 1), dtype=torch.float64, device=S.device)
    _check(lib().bb_ge2val(ctypes.c_void_p(S.data_ptr()), int(m), int(n), int(m), int(nb), TREES[tree],
                           VARIANTS[variant], PRECS[prec], ctypes.c_void_p(sigma.data_ptr()),
                           ctypes.c_void_p(vt.data_ptr()), vt.numel(), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                           ctypes.byref(o), _stream_handle(stream)), "bb_ge2val")
    if check:
        st = poll_error(ws, stream)
        if st != 0:
            raise BidiagError(st, "ge2val pipeline")
    return sigma[:k]


TREE_NAMES = {v: k for k, v in TREES.items()}
VARIANT_NAMES = {v: k for k, v in VARIANTS.items()}


def tuned_config(m, n, prec="f64"):
    """(nb, tree, variant) the offline tuner chose for the size class of m x n."""
    nb, tr, var = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().bb_tuned_config(int(m), int(n), PRECS[prec], ctypes.byref(nb), ctypes.byref(tr),
                                 ctypes.byref(var)), "bb_tuned_config")
    return nb.value, TREE_NAMES[tr.value], VARIANT_NAMES[var.value]


def _per_matrix(x, count, table, dtype=np.int32):
    if x is None:
        return None
    if isinstance(x, (str, int, np.integer)):
        x = [x] * count
    return np.ascontiguousarray([table[v] if table else int(v) for v in x], dtype=dtype)


class BatchPlan:
    """Task graphs of a batch of independent reductions (bb_batch_*)."""

    def __init__(self, shapes, nb=None, tree=None, variant=None, prec="f64", **opts):
        self.shapes = [(int(m), int(n)) for m, n in shapes]
        count = len(self.shapes)
        self.m = np.ascontiguousarray([s[0] for s in self.shapes], dtype=np.int64)
        self.n = np.ascontiguousarray([s[1] for s in self.shapes], dtype=np.int64)
        self._nb = _per_matrix(nb, count, None)
        self._tree = _per_matrix(tree, count, TREES)
        self._var = _per_matrix(variant, count, VARIANTS)
        self.prec = prec
        self._opts = make_opts(**opts)
        ptr = lambda a: None if a is None else a.ctypes.data
        h = ctypes.c_void_p()
        _check(lib().bb_batch_create(ctypes.byref(h), count, ptr(self.m), ptr(self.n), ptr(self._nb),
                                     ptr(self._tree), ptr(self._var), PRECS[prec],
                                     ctypes.byref(self._opts)), "bb_batch_create")
        self._h = h

    def __len__(self):
        return len(self.shapes)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.bb_batch_destroy(h)
            self._h = None

    def workspace(self):
        vt, ws = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().bb_batch_workspace(self._h, ctypes.byref(vt), ctypes.byref(ws)),
               "bb_batch_workspace")
        return vt.value, ws.value

    def info(self, i) -> dict:
        nb, tr, var = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        off, nrec = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().bb_batch_info(self._h, int(i), ctypes.byref(nb), ctypes.byref(tr),
                                   ctypes.byref(var), ctypes.byref(off), ctypes.byref(nrec)),
               "bb_batch_info")
        return {"nb": nb.value, "tree": TREE_NAMES[tr.value], "variant": VARIANT_NAMES[var.value],
                "rec_offset": off.value, "nrec": nrec.value}

    def alloc(self, device=None):
        import torch
        vt_b, ws_b = self.workspace()
        dev = device if device is not None else torch.device("cuda")
        return (torch.empty(max(vt_b, 8), dtype=torch.uint8, device=dev),
                torch.empty(max(ws_b, 8), dtype=torch.uint8, device=dev))

    def execute(self, ptrs, ldas, vt, ws, stream=None):
        """ptrs, ldas: int64 CUDA tensors (device pointers and leading dimensions)."""
        _check(lib().bb_batch_execute(self._h, ctypes.c_void_p(ptrs.data_ptr()),
                                      ctypes.c_void_p(ldas.data_ptr()),
                                      ctypes.c_void_p(vt.data_ptr()), vt.numel(),
                                      ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                      _stream_handle(stream)), "bb_batch_execute")

    def poll_error(self, ws, stream=None) -> int:
        st = ctypes.c_int()
        _check(lib().bb_batch_poll_error(self._h, ctypes.c_void_p(ws.data_ptr()),
                                         _stream_handle(stream), ctypes.byref(st)),
               "bb_batch_poll_error")
        return st.value

    def last_kernel_ms(self) -> float:
        ms = ctypes.c_double()
        _check(lib().bb_batch_last_kernel_ms(self._h, ctypes.byref(ms)), "bb_batch_last_kernel_ms")
        return ms.value


def pack_batch(mats, device="cuda"):
    """Copy matrices (numpy or torch, m_i x n_i) column-major into one device
    buffer.  Returns (buf, ptrs, ldas, offsets): ptrs/ldas are int64 device
    tensors for BatchPlan.execute, offsets the element offset of each matrix
    (lda = m)."""
    import torch
    sizes = [int(A.shape[0]) * int(A.shape[1]) for A in mats]
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    # One spare element keeps the buffer non-empty; zeroed so that whole
    # buffers compare equal across runs.
    buf = torch.zeros(int(offsets[-1]) + 1, dtype=torch.float64, device=device)
    for A, o, sz in zip(mats, offsets, sizes):
        T = torch.as_tensor(A, dtype=torch.float64)
        buf[int(o):int(o) + sz].copy_(T.t().reshape(-1))
    base = buf.data_ptr()
    ptrs = torch.as_tensor(base + 8 * offsets[:-1], dtype=torch.int64).to(device)
    ldas = torch.as_tensor([int(A.shape[0]) for A in mats], dtype=torch.int64).to(device)
    return buf, ptrs, ldas, offsets


def unpack(buf, offsets, shapes, i):
    """Matrix i of a packed batch as an m x n view (column-major storage)."""
    m, n = shapes[i]
    o = int(offsets[i])
    return buf[o:o + m * n].view(n, m).t()


def _band_function():
    import torch

    class BandBidiag(torch.autograd.Function):
        """B = band(A) with the hand-written adjoint as backward: the gradient
        of any loss reaches A through the band entries of B (the other entries
        are identically zero)."""

        @staticmethod
        def forward(ctx, A, nb, tree, variant):
            m, n = A.shape
            plan = Plan(m, n, nb, tree, variant)
            S = to_colmajor(A.detach())
            vt, ws = plan.alloc(S.device)
            plan.execute(S, m, vt, ws)
            st = poll_error(ws)
            if st != 0:
                raise BidiagError(st, "device scheduler")
            ctx.plan, ctx.vt, ctx.S = plan, vt, S
            return S.t().clone()

        @staticmethod
        def backward(ctx, Bbar):
            n = ctx.plan.n
            Ab = ctx.plan.adjoint(ctx.S, ctx.plan.m, Bbar[:n, :n], ctx.vt, check=True)
            return Ab.to(Bbar.dtype), None, None, None

    return BandBidiag


_BandBidiag = None


def band_autograd(A, nb, tree="greedy", variant="rbidiag"):
    """Differentiable band form: returns B (m x n); B.backward / autograd use
    bidiag_band_adjoint."""
    global _BandBidiag
    if _BandBidiag is None:
        _BandBidiag = _band_function()
    return _BandBidiag.apply(A, nb, tree, variant)
