#!/usr/bin/env python3
"""Band-bidiagonalization throughput on one MI355X.

Workload: the tall graded matrix, 32768 x 2048, A = U diag(s) V^T with s
geometric from 1 to 1e-8 (seeded), tile nb = 128, reduced to band form by
R-BiDiag (QR(p,q) then the band reduction of R, Section 3.5) with the Greedy
tree by default.  One step = one full reduction of a fresh copy of A already
resident in HBM (the copy is inside the timed region).  GFLOP/s uses the
paper's operation count 4 n^2 (m - n/3) for both BiDiag and R-BiDiag
(Section 6.2).  Also reported: BiDiag / R-BiDiag x Greedy / Auto on the same
input, the roofline of the persistent kernel (HIP events on the launch
stream), and the FP64 oracle timed on host cores on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "band-bidiag GFLOP/s (4n²(m−n/3)/t), % MFMA peak, mixed/batched vs FP64 at err"
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_plan(bb, torch, plan, S0, m, steps, warmup):
    vt, ws = plan.alloc()
    S = torch.empty_like(S0)
    for w in range(warmup):
        S.copy_(S0)
        plan.execute(S, m, vt, ws)
        log("  warmup %d: %.2f ms" % (w, plan.last_kernel_ms()))
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
        log("  step %d: %.2f ms" % (k, kms[-1]))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = bb.poll_error(ws)
    if st != 0:
        raise RuntimeError("device scheduler error %d" % st)
    return (t1 - t0) * 1e3 / steps, kms, S


def measured_traffic(args, m, n, nb):
    """HBM bytes per launch of the persistent kernel from the committed PMC
    summary (FETCH_SIZE + WRITE_SIZE, calibrated on a copy of known size), for
    the configuration it was measured on and only while the kernel source is
    the one measured; else None."""
    import hashlib
    if (args.workload, m, n, nb, args.variant, args.tree, args.prec, args.sched) != \
            ("tall_graded", 32768, 2048, 128, "rbidiag", "greedy", "f64", "persistent"):
        return None
    here = os.path.dirname(os.path.abspath(__file__))
    summary = os.path.join(here, "profiles",
                           "persistent_kernel_tall_graded_32768x2048_nb128_rbidiag_greedy.md")
    src = os.path.join(here, "paper_1611_06892_amd", "csrc", "kernels.hip")
    try:
        fields = dict(line.split(": ", 1) for line in open(summary).read().splitlines()
                      if line.startswith(("traffic_bytes: ", "kernel_source_sha256_prefix: ")))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    if fields.get("kernel_source_sha256_prefix") != sha:
        return None
    return float(fields["traffic_bytes"])


def cpu_baseline(workloads):
    """The FP64 oracle on a bounded sample of the same workload."""
    import oracle
    m, n, nb = 4096, 2048, 128
    A, _ = workloads.graded(m, n, 1, 2, 1e-8)
    t0 = time.perf_counter()
    oracle.band_reduce(A, nb)
    dt = time.perf_counter() - t0
    return {"value": round(workloads.flops_bidiag(m, n) / dt / 1e9, 3), "unit": "GFLOP/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "4096 x 2048 graded matrix (same recipe, seeds 1/2), nb = 128, unblocked "
                      "FP64 BiDiag, %.1f s" % dt}


def bench_batch(args, bb, torch, np, workloads):
    """4096 matrices, m ~ U{64..1024}, n ~ U{32..m}, N(0,1) (seed 5), each with
    the tuned (nb, tree, variant) of its size class; one step = all of them,
    from fresh copies already in HBM."""
    cfg = workloads.CONFIGS["batch"]
    log("generating the batch")
    mats = workloads.batch_shapes(cfg["count"], cfg["seed"], cfg["mlo"], cfg["mhi"], cfg["nlo"])
    shapes = [A.shape for A in mats]
    plan = bb.BatchPlan(shapes, prec=args.prec, timing=True)
    buf, ptrs, ldas, offs = bb.pack_batch(mats)
    orig = buf.clone()
    vt, ws = plan.alloc()
    log("batch: %d matrices, records %.1f GB" % (len(mats), vt.numel() / 1e9))
    for w in range(args.warmup):
        buf.copy_(orig)
        plan.execute(ptrs, ldas, vt, ws)
        log("  warmup %d: %.2f ms" % (w, plan.last_kernel_ms()))
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        buf.copy_(orig)
        plan.execute(ptrs, ldas, vt, ws)
        kms.append(plan.last_kernel_ms())
        log("  step %d: %.2f ms" % (k, kms[-1]))
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    st = plan.poll_error(ws)
    if st != 0:
        raise RuntimeError("device scheduler error %d" % st)
    flops = sum(workloads.flops_bidiag(m, n) for m, n in shapes)
    actual, classes = 0.0, {}
    for i, (m, n) in enumerate(shapes):
        inf = plan.info(i)
        actual += (workloads.flops_rbidiag_actual(m, n) if inf["variant"] == "rbidiag"
                   else workloads.flops_bidiag(m, n))
        key = "nb%d/%s/%s" % (inf["nb"], inf["tree"], inf["variant"])
        classes[key] = classes.get(key, 0) + 1
    # correctness outside the timed region: band structure of every matrix,
    # orthogonal invariance of the Frobenius norm, and the singular values of
    # a sample against numpy's SVD of A
    log("checking")
    band_ok, fro_err, sig_err = True, 0.0, 0.0
    for i, A in enumerate(mats):
        B = bb.unpack(buf, offs, shapes, i).cpu().numpy()
        nb = plan.info(i)["nb"]
        ii = np.arange(B.shape[0])[:, None]
        jj = np.arange(B.shape[1])[None, :]
        band_ok &= bool(np.all(B[(jj < ii) | (jj > ii + nb)] == 0.0))
        nA = np.linalg.norm(A)
        fro_err = max(fro_err, abs(np.linalg.norm(B) - nA) / nA)
        if i % 256 == 0:
            sa = np.linalg.svd(A, compute_uv=False)
            sb = np.linalg.svd(B, compute_uv=False)
            sig_err = max(sig_err, float(np.max(np.abs(sa - sb)) / nA))
    kern_ms = float(np.mean(kms))
    peak = FP64_PEAK_TFLOPS if args.prec == "f64" else FP32_PEAK_TFLOPS
    achieved = actual / (kern_ms * 1e-3) / 1e12
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        done = 0.0
        for i, A in enumerate(mats[:64]):
            oracle.band_reduce(A, plan.info(i)["nb"])
            done += workloads.flops_bidiag(*A.shape)
            if time.perf_counter() - t0 > 15.0:
                break
        dt = time.perf_counter() - t0
        cpu = {"value": round(done / dt / 1e9, 3), "unit": "GFLOP/s", "cores": oracle.num_threads(),
               "kind": "oracle", "sample": "the first matrices of the batch until 15 s, "
               "unblocked FP64 BiDiag, %.1f s" % dt}
    out = {
        "metric": METRIC, "value": round(flops / (ms_step * 1e-3) / 1e9, 2), "unit": "GFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"f64": "f64", "f64_upd_f32": "f64 panels, f32 updates",
                  "f64_upd_split32": "f64 panels, split-f32 updates"}[args.prec],
        "data": "synthetic",
        "config": {"workload": "batch of %d matrices, m~U{%d..%d}, n~U{%d..m}, tuned nb/tree/variant"
                   % (cfg["count"], cfg["mlo"], cfg["mhi"], cfg["nlo"]),
                   "count": len(mats), "classes": classes, "prec": args.prec,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                     "kernel": "persistent_kernel<nb, %d> (all groups)" % bb.PRECS[args.prec],
                     "kernel_ms": round(kern_ms, 3), "algorithmic_flops": actual},
        "cpu_baseline": cpu,
        "check": {"band_exact": band_ok, "max_fro_rel_err": fro_err,
                  "max_sigma_err_rel_normA_sample": sig_err},
    }
    print(json.dumps(out), flush=True)


def bench_adjoint(args, bb, torch, np, workloads):
    """8192 x 1024 N(0,1) (seed 6), R-BiDiag Greedy, nb = 128, and the gradient
    of sum(W * B) over the band (W N(0,1), seed 7).  One step = forward
    reduction + adjoint, from a fresh copy of A already in HBM; HIP events on
    the launch stream time each part."""
    cfg = workloads.CONFIGS["adjoint"]
    m, n, nb = cfg["m"], cfg["n"], cfg["nb"]
    A = workloads.gaussian(m, n, cfg["seed"])
    W = torch.as_tensor(workloads.band_weights(n, nb, cfg["wseed"])).cuda()
    S0 = bb.to_colmajor(torch.from_numpy(A))
    plan = bb.Plan(m, n, nb, args.tree, "rbidiag", prec=args.prec)
    vt, ws = plan.alloc()
    aws = torch.empty(plan.adjoint_workspace(), dtype=torch.uint8, device="cuda")
    S = torch.empty_like(S0)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fw, bw = [], []
    Ab = None
    for k in range(args.warmup + args.steps):
        S.copy_(S0)
        ev[0].record()
        plan.execute(S, m, vt, ws)
        ev[1].record()
        Ab = plan.adjoint(S, m, W, vt, ws=aws)
        ev[2].record()
        torch.cuda.synchronize()
        if k >= args.warmup:
            fw.append(ev[0].elapsed_time(ev[1]))
            bw.append(ev[1].elapsed_time(ev[2]))
        log("  step %d: forward %.2f ms, adjoint %.2f ms" % (k, ev[0].elapsed_time(ev[1]),
                                                            ev[1].elapsed_time(ev[2])))
    st = bb.poll_error(ws)
    if st != 0:
        raise RuntimeError("device scheduler error %d" % st)
    Ag = Ab.cpu().numpy()
    check = {}
    if args.prec != "f64":
        # mixed forward: distance to the gradient of the FP64 forward (central
        # differences of a forward with FP32 rounding would measure its noise)
        p64 = bb.Plan(m, n, nb, args.tree, "rbidiag")
        v64, w64 = p64.alloc()
        S.copy_(S0)
        p64.execute(S, m, v64, w64)
        A64 = p64.adjoint(S, m, W, v64).cpu().numpy()
        check["rel_diff_to_f64_gradient"] = float(np.linalg.norm(Ag - A64) / np.linalg.norm(A64))
        del p64, v64, w64
    else:
        check["fd_max_err_rel_grad_norm"] = fd_check(A, Ag, W, plan, bb, torch, np, m, n)
    f_ms, b_ms = float(np.median(fw)), float(np.median(bw))
    flops = workloads.flops_bidiag(m, n)
    dtype = {"f64": "f64", "f64_upd_f32": "f64 panels, f32 updates; f64 adjoint",
             "f64_upd_split32": "f64 panels, split-f32 updates; f64 adjoint"}[args.prec]
    out = {
        "metric": METRIC, "value": round(flops / ((f_ms + b_ms) * 1e-3) / 1e9, 2), "unit": "GFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(f_ms + b_ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": "adjoint 8192x1024 nb=128 rbidiag %s, forward + gradient of "
                               "sum(W*B)" % args.tree, "m": m, "n": n, "nb": nb, "prec": args.prec,
                   "parallelism": "single GPU"},
        "forward_ms": round(f_ms, 3), "adjoint_ms": round(b_ms, 3),
        "adjoint_over_forward": round(b_ms / f_ms, 3),
        "check": check,
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def fd_check(A, Ag, W, plan, bb, torch, np, m, n):
    """Central differences of the forward in 4 random unit directions: the
    largest error relative to the gradient's norm."""
    def L(M):
        Sm = bb.to_colmajor(torch.from_numpy(M))
        v2, w2 = plan.alloc()
        plan.execute(Sm, m, v2, w2)
        return float(torch.sum(W * Sm.t()[:n]))
    rng = np.random.default_rng(8)
    h = 1e-6 * np.linalg.norm(A)
    fd_err = 0.0
    for _ in range(4):
        E = rng.standard_normal((m, n))
        E /= np.linalg.norm(E)
        fd = (L(A + h * E) - L(A - h * E)) / (2 * h)
        fd_err = max(fd_err, abs(fd - float(np.sum(Ag * E))) / np.linalg.norm(Ag))
    return fd_err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--variant", default="rbidiag", choices=["bidiag", "rbidiag"])
    ap.add_argument("--tree", default="greedy", choices=["flatts", "flattt", "greedy", "auto"])
    ap.add_argument("--sched", default="persistent", choices=["persistent", "levels"])
    ap.add_argument("--prec", default="f64", choices=["f64", "f64_upd_f32", "f64_upd_split32"])
    ap.add_argument("--workload", default="tall_graded",
                    choices=["tall_graded", "square_graded", "batch", "adjoint"])
    ap.add_argument("--nb", type=int, default=0, help="tile size (0: the workload's)")
    ap.add_argument("--m", type=int, default=0, help="rows (0: the workload's)")
    ap.add_argument("--n", type=int, default=0, help="columns (0: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(one GPU's share at its real shape is what --gpus 1 measures)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import paper_1611_06892_amd as bb
    import workloads

    if args.workload == "batch":
        return bench_batch(args, bb, torch, np, workloads)
    if args.workload == "adjoint":
        return bench_adjoint(args, bb, torch, np, workloads)
    cfg = workloads.CONFIGS[args.workload]
    m, n, nb = args.m or cfg["m"], args.n or cfg["n"], args.nb or cfg["nb"]
    log("generating %d x %d graded input" % (m, n))
    if m * n <= 2 ** 27:
        A, s = workloads.graded(m, n, *cfg["seeds"], cfg["smin"])
        normA = float(np.linalg.norm(A))
        S0 = bb.to_colmajor(torch.from_numpy(A))
    else:
        Ad, s = workloads.graded_device(m, n, *cfg["seeds"], cfg["smin"])
        normA = float(torch.linalg.norm(Ad))
        S0 = bb.to_colmajor(Ad)
        del Ad
    flops_metric = workloads.flops_bidiag(m, n)

    plan = bb.Plan(m, n, nb, args.tree, args.variant, prec=args.prec, sched=args.sched,
                   timing=True)
    log("timing %s/%s: %d warmup + %d steps" % (args.variant, args.tree, args.warmup, args.steps))
    ms_step, kms, S = time_plan(bb, torch, plan, S0, m, args.steps, args.warmup)
    value = flops_metric / (ms_step * 1e-3) / 1e9

    # Correctness of the timed result (outside the timed region): exact band
    # structure and the singular values of B against the prescribed ones.
    Bd = S.t()
    i = torch.arange(m, device=Bd.device)[:, None]
    j = torch.arange(n, device=Bd.device)[None, :]
    band_ok = bool(torch.all(Bd[(j < i) | (j > i + nb)] == 0.0).item())
    log("checking the band form")
    sig_err = sig_rel = None
    if n <= 4096:
        sB = np.linalg.svd(Bd[:n].cpu().numpy(), compute_uv=False)
    elif n <= 8192:
        sB = torch.linalg.svdvals(Bd[:n].contiguous()).cpu().numpy()
    else:
        sB = None     # dense SVD too slow here; the Frobenius norm is checked instead
    if sB is not None:
        sig_err = float(np.max(np.abs(sB - s)))
        sig_rel = float(np.max(np.abs(sB - s) / s))
    fro_rel = abs(float(torch.linalg.norm(Bd)) - float(np.linalg.norm(s))) / float(np.linalg.norm(s))
    del Bd

    kern_ms = float(np.mean(kms))
    algo = workloads.flops_rbidiag_actual(m, n) if args.variant == "rbidiag" else flops_metric
    achieved = algo / (kern_ms * 1e-3) / 1e12
    peak = FP64_PEAK_TFLOPS if args.prec == "f64" else FP32_PEAK_TFLOPS
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                "traffic": measured_traffic(args, m, n, nb),
                "kernel": "persistent_kernel<%d, %d>" % (nb, bb.PRECS[args.prec]),
                "kernel_ms": round(kern_ms, 3),
                "algorithmic_flops": algo}

    variants = {}
    if not args.no_variants and args.workload == "tall_graded" and args.prec == "f64":
        for var in ("bidiag", "rbidiag"):
            for tree in ("greedy", "auto"):
                p2 = bb.Plan(m, n, nb, tree, var, sched=args.sched, timing=True)
                ms2, _, _ = time_plan(bb, torch, p2, S0, m, 2, 1)
                variants["%s/%s" % (var, tree)] = round(flops_metric / (ms2 * 1e-3) / 1e9, 1)
                del p2
    cpu = None if (args.no_cpu_baseline or args.workload != "tall_graded") else cpu_baseline(workloads)

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"f64": "f64", "f64_upd_f32": "f64 panels, f32 updates",
                  "f64_upd_split32": "f64 panels, split-f32 updates"}[args.prec],
        "data": "synthetic",
        "config": {"workload": "%s %dx%d nb=%d %s %s" % (args.workload, m, n, nb, args.variant,
                                                          args.tree),
                   "m": m, "n": n, "nb": nb, "variant": args.variant, "tree": args.tree,
                   "sched": args.sched, "prec": args.prec, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "variants_gflops": variants,
        "check": {"band_exact": band_ok, "max_abs_sigma_err": sig_err,
                  "max_rel_sigma_err": sig_rel, "fro_norm_rel_err": fro_rel,
                  "sigma_tol": 50 * n * np.finfo(np.float64).eps * normA},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
