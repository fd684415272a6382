#!/usr/bin/env python3
"""Band-bidiagonalization throughput on one MI355X.

Headline workload: the square graded matrix, 16384 x 16384, A = U diag(s) V^T
with s geometric from 1 to 1e-6 (seeded), tile nb = 256, reduced to band form
by BiDiag (Section 3.4) with the Auto tree, FP64.  One step = one full
reduction of a fresh copy of A already resident in HBM (the copy is inside the
timed region).  GFLOP/s uses the paper's operation count 4 n^2 (m - n/3)
(Section 6.2).  The line also carries the roofline of the persistent kernel
(HIP events on its launch stream), the FP64 oracle timed on host cores on a
bounded sample of the same recipe (all cores and one thread), and extra keys
for the other workloads: the singular values of the square input through the
band (GE2VAL: bulge chase and bisection after the reduction, at the headline
nb and at nb = 128), the tall graded 32768 x 2048 reduction, the batch of 4096
matrices, the adjoint of the 8192 x 1024 reduction, the same square at
nb = 128 and its FP32-update form.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ...]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

METRIC = "band-bidiag GFLOP/s (4n²(m−n/3)/t), % MFMA peak, mixed/batched vs FP64 at err"
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
HERE = os.path.dirname(os.path.abspath(__file__))
DTYPES = {"f64": "f64", "f64_upd_f32": "f64 panels, f32 updates",
          "f64_upd_split32": "f64 panels, split-f32 updates"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_plan(bb, torch, plan, S0, m, steps, warmup, label=""):
    """Warmup, then `steps` timed reductions of fresh copies of S0.
    Returns (wall ms per step, kernel ms per step list, the reduced copy)."""
    vt, ws = plan.alloc()
    S = torch.empty_like(S0)
    for w in range(warmup):
        S.copy_(S0)
        plan.execute(S, m, vt, ws)
        log("  %s warmup %d: %.2f ms" % (label, w, plan.last_kernel_ms()))
    if warmup:      # the status word is written by an execution; before one it is undefined
        st = bb.poll_error(ws)
        if st != 0:
            raise RuntimeError("device scheduler error %d" % st)
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for k in range(steps):
        S.copy_(S0)
        plan.execute(S, m, vt, ws)
        kms.append(plan.last_kernel_ms())
        log("  %s step %d: %.2f ms" % (label, k, kms[-1]))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = bb.poll_error(ws)
    if st != 0:
        raise RuntimeError("device scheduler error %d" % st)
    return (t1 - t0) * 1e3 / steps, kms, S, vt


def measured_traffic(workload, m, n, nb, variant, tree, prec):
    """HBM bytes per launch of the persistent kernel from the committed PMC
    summary of this configuration (FETCH_SIZE + WRITE_SIZE, calibrated on a
    copy of known size), only while the kernel source is the one measured;
    else None."""
    name = "persistent_kernel_%s_%dx%d_nb%d_%s_%s.md" % (workload, m, n, nb, variant, tree)
    if prec != "f64":
        return None
    summary = os.path.join(HERE, "profiles", name)
    src = os.path.join(HERE, "paper_1611_06892_amd", "csrc", "kernels.hip")
    try:
        fields = dict(line.split(": ", 1) for line in open(summary).read().splitlines()
                      if line.startswith(("traffic_bytes: ", "kernel_source_sha256_prefix: ")))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    if fields.get("kernel_source_sha256_prefix") != sha or "traffic_bytes" not in fields:
        return None
    return float(fields["traffic_bytes"])


ORACLE_SNIPPET = r"""
import sys, time, json
sys.path.insert(0, %r)
import oracle, workloads
m, n, nb, seeds, smin = %d, %d, %d, (%d, %d), %r
A, _ = workloads.graded(m, n, seeds[0], seeds[1], smin)
t0 = time.perf_counter()
oracle.band_reduce(A, nb)
dt = time.perf_counter() - t0
print(json.dumps({"seconds": dt, "threads": oracle.num_threads(),
                  "gflops": workloads.flops_bidiag(m, n) / dt / 1e9}))
"""


def oracle_rate(m, n, nb, seeds, smin, threads=None):
    """The oracle (unblocked FP64 BiDiag) on one graded m x n matrix, in a
    child process so that the OpenMP thread count can be set."""
    env = dict(os.environ)
    if threads is not None:
        env["OMP_NUM_THREADS"] = str(threads)
    code = ORACLE_SNIPPET % (HERE, m, n, nb, seeds[0], seeds[1], smin)
    out = subprocess.check_output([sys.executable, "-c", code], env=env)
    return json.loads(out.decode().strip().splitlines()[-1])


ORACLE_CFG_SNIPPET = r"""
import sys, time, json
sys.path.insert(0, %r)
import oracle, workloads
m, n, nb, variant, kind, seeds, smin = %d, %d, %d, %r, %r, (%d, %d), %r
if kind == "graded":
    A, _ = workloads.graded(m, n, seeds[0], seeds[1], smin)
else:
    A = workloads.gaussian(m, n, seeds[0])
t0 = time.perf_counter()
if variant == "rbidiag":
    oracle.rbidiag_reduce(A, nb)
else:
    oracle.band_reduce(A, nb)
dt = time.perf_counter() - t0
print(json.dumps({"seconds": dt, "threads": oracle.num_threads(),
                  "gflops": workloads.flops_bidiag(m, n) / dt / 1e9}))
"""


def oracle_cfg_rate(m, n, nb, variant, kind, seeds, smin=0.0, threads=None):
    """The oracle on one m x n matrix of a workload's recipe (gaussian or
    graded; BiDiag or R-BiDiag), in a child process so that the OpenMP thread
    count can be set; GFLOP/s with the metric count 4n^2(m - n/3)."""
    env = dict(os.environ)
    if threads is not None:
        env["OMP_NUM_THREADS"] = str(threads)
    code = ORACLE_CFG_SNIPPET % (HERE, m, n, nb, variant, kind, seeds[0], seeds[1], smin)
    out = subprocess.check_output([sys.executable, "-c", code], env=env)
    r = json.loads(out.decode().strip().splitlines()[-1])
    return {"gflops": round(r["gflops"], 3), "seconds": round(r["seconds"], 2), "cores": r["threads"]}


def cpu_oracle_configs():
    """The oracle on the other workloads' recipes: the 512 x 512 N(0,1) square
    (nb = 64, BiDiag) in full at all cores and one thread, the 8192 x 1024
    N(0,1) adjoint workload's forward (nb = 128, R-BiDiag) in full at all
    cores, and a 4096 x 2048 sample of the tall graded recipe (nb = 128,
    R-BiDiag) at all cores."""
    import oracle
    oracle.build()
    return {
        "small_square_512x512_nb64_bidiag": {
            "all_cores": oracle_cfg_rate(512, 512, 64, "bidiag", "gaussian", (0, 0)),
            "one_thread": oracle_cfg_rate(512, 512, 64, "bidiag", "gaussian", (0, 0), threads=1)},
        "adjoint_forward_8192x1024_nb128_rbidiag": {
            "all_cores": oracle_cfg_rate(8192, 1024, 128, "rbidiag", "gaussian", (6, 0))},
        "tall_graded_sample_4096x2048_nb128_rbidiag": {
            "all_cores": oracle_cfg_rate(4096, 2048, 128, "rbidiag", "graded", (1, 2), 1e-8)},
    }


def cpu_baseline_square():
    """The oracle on bounded samples of the square graded recipe (nb = 256):
    2048 x 2048 on all host cores, 1024 x 1024 on one thread."""
    import oracle
    oracle.build()
    allc = oracle_rate(2048, 2048, 256, (3, 4), 1e-6)
    one = oracle_rate(1024, 1024, 256, (3, 4), 1e-6, threads=1)
    return {"value": round(allc["gflops"], 3), "unit": "GFLOP/s", "cores": allc["threads"],
            "kind": "oracle",
            "sample": "2048 x 2048 graded matrix of the same recipe (seeds 3/4, s 1..1e-6), nb = 256, "
                      "unblocked FP64 BiDiag, %.1f s on %d threads" % (allc["seconds"], allc["threads"]),
            "single_thread": {"value": round(one["gflops"], 3), "unit": "GFLOP/s", "cores": 1,
                              "sample": "1024 x 1024 of the same recipe, nb = 256, %.1f s"
                                        % one["seconds"]}}


def graded_input(bb, torch, np, workloads, m, n, seeds, smin):
    if m * n <= 2 ** 27:
        A, s = workloads.graded(m, n, *seeds, smin)
        Ad = torch.from_numpy(A).cuda()
    else:
        Ad, s = workloads.graded_device(m, n, *seeds, smin)
    return Ad, s


def gaussian_input(torch, m, n, seed):
    """m x n N(0,1) on the device from a seeded torch generator.  The
    reduction's memory accesses do not depend on the values, so this input
    stands in for the graded one where its generation (a device QR) cannot
    run, as under hardware-counter collection."""
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    return torch.randn(m, n, generator=gen, device="cuda", dtype=torch.float64)


def chase_bytes(n, nb):
    """Algorithmic bytes of the bulge chase: every step reads and writes once
    the entries its two reflectors change (the cleared row's block, the
    rows between it and the diagonal block, the diagonal block and the block
    right of it), 16 bytes an entry."""
    total = 0
    for k in range(max(n - 2, 0) if nb > 1 else 0):
        c = k + 1
        first = True
        while c < n:
            L = min(nb, n - c)
            Lq = max(min(nb, n - c - nb), 0)
            rows_above = 1 if first else nb            # rows rr .. c-1
            total += (rows_above * L + L * L + L * Lq) * 16
            c += nb
            first = False
    return total


def chase_traffic(n, nb):
    """HBM bytes of one bulge chase (n, nb) from the committed PMC summary
    (FETCH_SIZE + WRITE_SIZE, calibrated on a copy of known size), only while
    the chase's source is the one measured; else None."""
    summary = os.path.join(HERE, "profiles", "chase_kernel_traffic_square_%d.md" % n)
    src = os.path.join(HERE, "paper_1611_06892_amd", "csrc", "ge2val.hip")
    key = "traffic_bytes_nb%d" % nb
    try:
        fields = dict(line.split(": ", 1) for line in open(summary).read().splitlines()
                      if line.startswith((key + ": ", "kernel_source_sha256_prefix: ")))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    if fields.get("kernel_source_sha256_prefix") != sha or key not in fields:
        return None
    return float(fields[key])


def ge2val_stage(bb, torch, np, S, m, n, nb, s_ref, e2bnd_ms):
    """BND2BD + BD2VAL on the band a reduction left in S (column-major, leading
    dimension m), timed with HIP events on the launch stream; singular values
    checked against the prescribed ones (when the input has them)."""
    warm = torch.zeros(300, 300, dtype=torch.float64, device="cuda")
    bb.bd2val(*bb.bnd2bd(warm, 300, 300, min(nb, 299)))           # code objects loaded before timing
    ws = torch.empty(bb.bnd2bd_workspace(n, nb), dtype=torch.uint8, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    ev[0].record()
    d, e = bb.bnd2bd(S, m, n, nb, ws=ws, watchdog_s=60.0, check=False)
    ev[1].record()
    sig = bb.bd2val(d, e)
    ev[2].record()
    torch.cuda.synchronize()
    st = bb.poll_error(ws)
    if st != 0:
        raise RuntimeError("bulge chase error %d" % st)
    chase_ms = ev[0].elapsed_time(ev[1])
    bd_ms = ev[1].elapsed_time(ev[2])
    err = None
    if s_ref is not None:
        ref = np.sort(np.asarray(s_ref))[::-1]
        err = float(np.max(np.abs(sig.cpu().numpy() - ref))) / float(ref[0])
    nbytes = chase_bytes(n, nb)
    gbs = nbytes / (chase_ms * 1e-3) / 1e9
    return {"nb": nb, "ge2bnd_ms": round(e2bnd_ms, 3), "bnd2bd_ms": round(chase_ms, 3),
            "bd2val_ms": round(bd_ms, 3), "total_ms": round(e2bnd_ms + chase_ms + bd_ms, 3),
            "sigma_max_rel_err": err, "tol": 50 * n * np.finfo(np.float64).eps,
            "bnd2bd_roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": 8000.0, "unit": "GB/s",
                                "frac": round(gbs / 8000.0, 5), "traffic": chase_traffic(n, nb),
                                "kernel": "chase_kernel<%s>" % ("true" if nb <= 64 else "false"),
                                "algorithmic_bytes": nbytes}}


def bench_square(args, bb, torch, np, workloads, nb=None, tree=None, prec=None, steps=None,
                 warmup=None, probes=True, label="square", ge2val=False):
    """The graded m x n square workload (default 16384^2): reduction timing,
    band check, ||B||_F against ||s||, probe vectors through Q and P."""
    cfg = workloads.CONFIGS["square_graded"]
    m, n = args.m or cfg["m"], args.n or cfg["n"]
    nb = nb or args.nb or cfg["nb"]
    tree = tree or args.tree
    prec = prec or args.prec
    variant = args.variant
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    log("generating %d x %d %s input" % (m, n, args.input))
    if args.input == "gaussian":
        Ad = gaussian_input(torch, m, n, cfg["seeds"][0])
        s = None
    else:
        Ad, s = graded_input(bb, torch, np, workloads, m, n, cfg["seeds"], cfg["smin"])
    nA = float(torch.linalg.norm(Ad))
    ref = nA if s is None else float(np.linalg.norm(s))
    S0 = bb.to_colmajor(Ad)
    plan = bb.Plan(m, n, nb, tree, variant, prec=prec, sched=args.sched, timing=True,
                   watchdog_s=60.0)
    log("timing %s %s/%s nb=%d %s: %d warmup + %d steps" % (label, variant, tree, nb, prec, warmup, steps))
    ms_step, kms, S, vt = time_plan(bb, torch, plan, S0, m, steps, warmup, label)
    B = S.t()
    i = torch.arange(m, device=B.device)[:, None]
    j = torch.arange(n, device=B.device)[None, :]
    band_ok = bool(torch.all(B[(j < i) | (j > i + nb)] == 0.0).item())
    fro = abs(float(torch.linalg.norm(B)) - ref) / ref
    probe = None
    if probes:
        gen = torch.Generator(device="cuda")
        gen.manual_seed(11)
        X = torch.randn(n, 8, generator=gen, device="cuda", dtype=torch.float64)
        Y1 = Ad @ X
        Xs = X.t().contiguous()
        plan.apply_p(Xs, n, 8, vt, transpose=True)
        Zs = (B @ Xs.t()).t().contiguous()
        plan.apply_q(Zs, m, 8, vt)
        torch.cuda.synchronize()
        probe = float(torch.linalg.norm(Y1 - Zs.t())) / (nA * float(torch.linalg.norm(X)))
    kern_ms = float(np.mean(kms))
    g2v = None
    if ge2val:
        log("GE2VAL: band to bidiagonal and singular values at nb=%d" % nb)
        g2v = [ge2val_stage(bb, torch, np, S, m, n, nb, s, kern_ms)]
        del S, B, vt
        nb2 = 128
        plan2 = bb.Plan(m, n, nb2, "greedy", variant, sched=args.sched, timing=True, watchdog_s=60.0)
        vt2, ws2 = plan2.alloc()
        S2 = S0.clone()
        plan2.execute(S2, m, vt2, ws2)
        torch.cuda.synchronize()
        if bb.poll_error(ws2) != 0:
            raise RuntimeError("device scheduler error %d" % bb.poll_error(ws2))
        log("GE2VAL: the same input reduced at nb=%d: %.2f ms" % (nb2, plan2.last_kernel_ms()))
        g2v.append(ge2val_stage(bb, torch, np, S2, m, n, nb2, s, plan2.last_kernel_ms()))
        del S2, vt2, ws2
    else:
        del S, B
    del Ad, S0
    flops = workloads.flops_bidiag(m, n)
    algo = workloads.flops_rbidiag_actual(m, n) if variant == "rbidiag" else flops
    peak = FP64_PEAK_TFLOPS if prec == "f64" else FP32_PEAK_TFLOPS
    achieved = algo / (kern_ms * 1e-3) / 1e12
    return {
        "m": m, "n": n, "nb": nb, "variant": variant, "tree": tree, "prec": prec,
        "ms_per_step": ms_step, "kernel_ms": kern_ms, "gflops": flops / (ms_step * 1e-3) / 1e9,
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4),
                     "traffic": measured_traffic("square_graded", m, n, nb, variant, tree, prec),
                     "kernel": "persistent_kernel<%d, %d>" % (nb, bb.PRECS[prec]),
                     "kernel_ms": round(kern_ms, 3), "algorithmic_flops": algo},
        "check": {"band_exact": band_ok, "fro_norm_rel_err": fro, "probe_rel_err": probe,
                  "tol": 50 * n * np.finfo(np.float64).eps},
        "ge2val": g2v,
    }


def bench_tall(args, bb, torch, np, workloads, steps=5, warmup=2, variant="rbidiag", tree="greedy"):
    """32768 x 2048 graded (s 1 .. 1e-8), nb = 128."""
    cfg = workloads.CONFIGS["tall_graded"]
    m, n, nb = cfg["m"], cfg["n"], cfg["nb"]
    log("generating %d x %d graded input" % (m, n))
    Ad, s = graded_input(bb, torch, np, workloads, m, n, cfg["seeds"], cfg["smin"])
    S0 = bb.to_colmajor(Ad)
    del Ad
    plan = bb.Plan(m, n, nb, tree, variant, timing=True)
    ms_step, kms, S, _ = time_plan(bb, torch, plan, S0, m, steps, warmup, "tall")
    sB = np.linalg.svd(S.t()[:n].cpu().numpy(), compute_uv=False)
    kern_ms = float(np.mean(kms))
    flops = workloads.flops_bidiag(m, n)
    algo = workloads.flops_rbidiag_actual(m, n) if variant == "rbidiag" else flops
    return {"workload": "tall_graded %dx%d nb=%d %s %s" % (m, n, nb, variant, tree),
            "gflops": round(flops / (ms_step * 1e-3) / 1e9, 2), "ms_per_step": round(ms_step, 3),
            "kernel_ms": round(kern_ms, 3),
            "frac_fp64_peak": round(algo / (kern_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4),
            "max_abs_sigma_err": float(np.max(np.abs(sB - s)))}


def bench_batch(args, bb, torch, np, workloads, steps=3, warmup=1, prec="f64"):
    """4096 matrices, m ~ U{64..1024}, n ~ U{32..m}, N(0,1) (seed 5), each with
    the tuned (nb, tree, variant) of its size class."""
    cfg = workloads.CONFIGS["batch"]
    log("generating the batch")
    mats = workloads.batch_shapes(cfg["count"], cfg["seed"], cfg["mlo"], cfg["mhi"], cfg["nlo"])
    shapes = [A.shape for A in mats]
    plan = bb.BatchPlan(shapes, prec=prec, timing=True)
    buf, ptrs, ldas, offs = bb.pack_batch(mats)
    orig = buf.clone()
    vt, ws = plan.alloc()
    for w in range(warmup):
        buf.copy_(orig)
        plan.execute(ptrs, ldas, vt, ws)
        log("  batch warmup %d: %.2f ms" % (w, plan.last_kernel_ms()))
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for k in range(steps):
        buf.copy_(orig)
        plan.execute(ptrs, ldas, vt, ws)
        kms.append(plan.last_kernel_ms())
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / steps
    if plan.poll_error(ws) != 0:
        raise RuntimeError("device scheduler error in the batch")
    flops = sum(workloads.flops_bidiag(m, n) for m, n in shapes)
    band_ok, fro_err = True, 0.0
    for i, A in enumerate(mats):
        B = bb.unpack(buf, offs, shapes, i).cpu().numpy()
        nb = plan.info(i)["nb"]
        ii = np.arange(B.shape[0])[:, None]
        jj = np.arange(B.shape[1])[None, :]
        band_ok &= bool(np.all(B[(jj < ii) | (jj > ii + nb)] == 0.0))
        nA = np.linalg.norm(A)
        fro_err = max(fro_err, abs(np.linalg.norm(B) - nA) / nA)
    del buf, orig, vt, ws
    return {"workload": "batch of %d matrices, m~U{%d..%d}, n~U{%d..m}, tuned nb/tree/variant, %s"
                        % (cfg["count"], cfg["mlo"], cfg["mhi"], cfg["nlo"], prec),
            "gflops": round(flops / (ms_step * 1e-3) / 1e9, 2), "ms_per_step": round(ms_step, 3),
            "kernel_ms": round(float(np.mean(kms)), 3), "band_exact": band_ok,
            "max_fro_rel_err": fro_err}


def bench_adjoint(args, bb, torch, np, workloads, steps=3, warmup=1):
    """8192 x 1024 N(0,1) (seed 6), R-BiDiag Greedy, nb = 128: forward plus the
    gradient of sum(W * B) over the band (W N(0,1), seed 7)."""
    cfg = workloads.CONFIGS["adjoint"]
    m, n, nb = cfg["m"], cfg["n"], cfg["nb"]
    A = workloads.gaussian(m, n, cfg["seed"])
    W = torch.as_tensor(workloads.band_weights(n, nb, cfg["wseed"])).cuda()
    S0 = bb.to_colmajor(torch.from_numpy(A))
    plan = bb.Plan(m, n, nb, "greedy", "rbidiag")
    vt, ws = plan.alloc()
    aws = torch.empty(plan.adjoint_workspace(), dtype=torch.uint8, device="cuda")
    S = torch.empty_like(S0)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fw, bw = [], []
    for k in range(warmup + steps):
        S.copy_(S0)
        ev[0].record()
        plan.execute(S, m, vt, ws)
        ev[1].record()
        plan.adjoint(S, m, W, vt, ws=aws)
        ev[2].record()
        torch.cuda.synchronize()
        if k >= warmup:
            fw.append(ev[0].elapsed_time(ev[1]))
            bw.append(ev[1].elapsed_time(ev[2]))
    if bb.poll_error(ws) != 0 or plan.adjoint_poll_error(aws) != 0:
        raise RuntimeError("device scheduler error in the adjoint")
    f_ms, b_ms = float(np.median(fw)), float(np.median(bw))
    return {"workload": "adjoint 8192x1024 nb=128 rbidiag greedy, forward + gradient of sum(W*B)",
            "forward_ms": round(f_ms, 3), "adjoint_ms": round(b_ms, 3),
            "adjoint_over_forward": round(b_ms / f_ms, 3),
            "gflops_forward": round(workloads.flops_bidiag(m, n) / (f_ms * 1e-3) / 1e9, 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="square_graded", choices=["square_graded"])
    ap.add_argument("--variant", default="bidiag", choices=["bidiag", "rbidiag", "threestep"])
    ap.add_argument("--tree", default="auto", choices=["flatts", "flattt", "greedy", "auto"])
    ap.add_argument("--sched", default="persistent", choices=["persistent", "levels"])
    ap.add_argument("--prec", default="f64", choices=["f64", "f64_upd_f32", "f64_upd_split32"])
    ap.add_argument("--nb", type=int, default=0, help="tile size (0: the workload's)")
    ap.add_argument("--m", type=int, default=0, help="rows (0: the workload's)")
    ap.add_argument("--n", type=int, default=0, help="columns (0: the workload's)")
    ap.add_argument("--extras", default="ge2val,tall,batch,adjoint,nb128,f32",
                    help="comma list of extra workloads (empty: none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--input", default="graded", choices=["graded", "gaussian"],
                    help="entries of the square workload: graded singular values (the workload), or "
                         "N(0,1) of the same shape (same memory accesses; no device QR to build it)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(one GPU's share at its real shape is what --gpus 1 measures)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    sys.path.insert(0, HERE)
    import paper_1611_06892_amd as bb
    import workloads

    wanted = [e for e in args.extras.split(",") if e]
    head = bench_square(args, bb, torch, np, workloads, ge2val="ge2val" in wanted)
    extras = {}
    if head["ge2val"]:
        extras["ge2val"] = {"workload": "GE2BND + BND2BD + BD2VAL of the square graded %dx%d input, "
                                        "the headline band and one reduced at nb=128 (greedy tree)"
                                        % (head["m"], head["n"]),
                            "runs": head["ge2val"]}
    if "nb128" in wanted:
        r = bench_square(args, bb, torch, np, workloads, nb=128, tree="greedy", prec="f64", steps=3,
                         warmup=1, probes=False, label="square nb128")
        extras["square_nb128_greedy"] = {"gflops": round(r["gflops"], 2), "kernel_ms": round(r["kernel_ms"], 3),
                                         "frac_fp64_peak": r["roofline"]["frac"],
                                         "fro_norm_rel_err": r["check"]["fro_norm_rel_err"]}
    if "f32" in wanted:
        r = bench_square(args, bb, torch, np, workloads, prec="f64_upd_f32", steps=3, warmup=1,
                         probes=False, label="square f32 updates")
        extras["square_f32_updates"] = {"gflops": round(r["gflops"], 2), "kernel_ms": round(r["kernel_ms"], 3),
                                        "speed_vs_f64": round(head["kernel_ms"] / r["kernel_ms"], 3),
                                        "fro_norm_rel_err": r["check"]["fro_norm_rel_err"]}
    if "tall" in wanted:
        extras["tall_graded"] = bench_tall(args, bb, torch, np, workloads)
    if "adjoint" in wanted:
        extras["adjoint"] = bench_adjoint(args, bb, torch, np, workloads)
    if "batch" in wanted:
        extras["batch"] = bench_batch(args, bb, torch, np, workloads)
    cpu = None if args.no_cpu_baseline else cpu_baseline_square()
    if not args.no_cpu_baseline:
        extras["cpu_oracle_other_workloads"] = cpu_oracle_configs()

    out = {
        "metric": METRIC, "value": round(head["gflops"], 2), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(head["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPES[head["prec"]], "data": "synthetic",
        "config": {"workload": "square_%s %dx%d nb=%d %s %s" % (args.input, head["m"], head["n"], head["nb"],
                                                               head["variant"], head["tree"]),
                   "m": head["m"], "n": head["n"], "nb": head["nb"], "variant": head["variant"],
                   "tree": head["tree"], "sched": args.sched, "prec": head["prec"],
                   "parallelism": "single GPU"},
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "check": head["check"],
        "extras": extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
