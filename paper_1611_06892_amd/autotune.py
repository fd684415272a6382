"""Offline tuner of the batched reduction: for each size class of matrices,
time every (nb, tree, variant) candidate as a batch on the GPU and keep the
fastest (batch throughput, 4 n^2 (m - n/3) flops per matrix).

Writes the table compiled into the library (csrc/tuned_table.inc format) and a
readable summary.  Run on the target GPU, then copy the table into csrc/ and
rebuild:

    python -m paper_1611_06892_amd.autotune --out-dir gpurun_out/tune

Classes: rows m in [64,192), [192,384), [384,640), [640,1025) crossed with the
aspect 1000 n/m in (0,250], (250,500], (500,1000].  Each class is sampled by
seeded N(0,1) matrices with (m, n) uniform inside the class; the sample holds
at least 256 matrices and about 2e10 flop (at most 1024 matrices), so that
every candidate runs in the throughput regime of a large batch.
"""
from __future__ import annotations

import argparse
import itertools
import os
import sys

import numpy as np

M_EDGES = [64, 192, 384, 640, 1025]
R_EDGES = [0, 250, 500, 1000]
NBS = [32, 64, 128]
TREES = ["greedy", "flatts", "flattt", "auto"]
VARIANTS = ["bidiag", "rbidiag"]
TARGET_FLOPS = 2.0e10
MIN_COUNT = 256          # enough matrices to occupy every CU, as in a large batch
MAX_COUNT = 1024


def log(*a):
    print(*a, flush=True)


def class_sample(ci, ri, seed):
    rng = np.random.default_rng(seed)
    m_lo, m_hi = M_EDGES[ci], M_EDGES[ci + 1]
    r_lo, r_hi = R_EDGES[ri], R_EDGES[ri + 1]
    shapes, flops = [], 0.0
    while (flops < TARGET_FLOPS or len(shapes) < MIN_COUNT) and len(shapes) < MAX_COUNT:
        m = int(rng.integers(m_lo, m_hi))
        n_lo = max(1, (r_lo * m) // 1000 + 1)
        n_hi = max(n_lo, (r_hi * m) // 1000)
        n = int(rng.integers(n_lo, n_hi + 1))
        shapes.append((m, n))
        flops += 4.0 * n * n * (m - n / 3.0)
    mats = [np.asfortranarray(rng.standard_normal(s)) for s in shapes]
    return shapes, mats, flops


def time_candidate(bb, torch, shapes, orig, ptrs, ldas, work, nb, tree, variant, reps=2):
    plan = bb.BatchPlan(shapes, nb=nb, tree=tree, variant=variant, timing=True, watchdog_s=30.0)
    vt, ws = plan.alloc()
    best = float("inf")
    for r in range(reps + 1):
        work.copy_(orig)
        plan.execute(ptrs, ldas, vt, ws)
        ms = plan.last_kernel_ms()
        if r > 0:
            best = min(best, ms)
    st = plan.poll_error(ws)
    if st != 0:
        raise RuntimeError("device scheduler error %d" % st)
    del vt, ws, plan
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out-dir", default="gpurun_out/tune")
    ap.add_argument("--seed", type=int, default=2024)
    args = ap.parse_args()
    import torch
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import paper_1611_06892_amd as bb

    os.makedirs(args.out_dir, exist_ok=True)
    rows, report = [], []
    for ci, ri in itertools.product(range(len(M_EDGES) - 1), range(len(R_EDGES) - 1)):
        shapes, mats, flops = class_sample(ci, ri, args.seed + 10 * ci + ri)
        buf, ptrs, ldas, _ = bb.pack_batch(mats)
        orig = buf.clone()
        log("class m[%d,%d) r(%d,%d]: %d matrices, %.2e flop" %
            (M_EDGES[ci], M_EDGES[ci + 1], R_EDGES[ri], R_EDGES[ri + 1], len(shapes), flops))
        results = []
        for nb, tree, variant in itertools.product(NBS, TREES, VARIANTS):
            ms = time_candidate(bb, torch, shapes, orig, ptrs, ldas, buf, nb, tree, variant)
            gf = flops / (ms * 1e-3) / 1e9
            results.append((gf, ms, nb, tree, variant))
            log("  nb %3d %-7s %-8s %8.2f ms %8.1f GFLOP/s" % (nb, tree, variant, ms, gf))
        results.sort(reverse=True)
        gf, ms, nb, tree, variant = results[0]
        m_hi = M_EDGES[ci + 1] if ci + 2 < len(M_EDGES) else 1 << 30
        rows.append((M_EDGES[ci] if ci > 0 else 0, m_hi, R_EDGES[ri], R_EDGES[ri + 1], nb,
                     bb.TREES[tree], bb.VARIANTS[variant]))
        report.append((M_EDGES[ci], M_EDGES[ci + 1], R_EDGES[ri], R_EDGES[ri + 1], len(shapes),
                       results[:3], results[-1]))
        del buf, orig, ptrs, ldas
        torch.cuda.empty_cache()

    inc = ["// (nb, tree, variant) per size class for matrices of a batch.  Written by",
           "// paper_1611_06892_amd/autotune.py from measurements; edit by re-running it.",
           "// Columns: m_lo, m_hi (rows in [m_lo, m_hi)), r_lo, r_hi (1000 n / m in",
           "// (r_lo, r_hi]), nb, tree (BB_FLATTS..BB_AUTO), variant (BB_BIDIAG/RBIDIAG).",
           "static const int kTunedTable[][7] = {"]
    for r in rows:
        inc.append("    {%d, %s, %d, %d, %d, %d, %d}," %
                   (r[0], "1 << 30" if r[1] == 1 << 30 else str(r[1]), r[2], r[3], r[4], r[5], r[6]))
    inc.append("};")
    with open(os.path.join(args.out_dir, "tuned_table.inc"), "w") as f:
        f.write("\n".join(inc) + "\n")
    md = ["# Batched reduction: tuned (nb, tree, variant) per size class",
          "",
          "Command: `python -m paper_1611_06892_amd.autotune --out-dir %s` (seed %d)." %
          (args.out_dir, args.seed),
          "Each class is a batch of seeded N(0,1) matrices with (m, n) uniform in the class, "
          "at least %d matrices and about %.0e flop (at most %d); time = best of 2 runs after one "
          "warm-up, HIP events around the batch's launches; GFLOP/s = sum 4n^2(m-n/3) / time." %
          (MIN_COUNT, TARGET_FLOPS, MAX_COUNT),
          "",
          "| m | 1000 n/m | matrices | best (GFLOP/s) | 2nd | 3rd | worst |",
          "|---|---|---|---|---|---|---|"]
    fmt = lambda r: "nb %d %s %s %.0f" % (r[2], r[3], r[4], r[0])
    for (m0, m1, r0, r1, cnt, top, worst) in report:
        md.append("| [%d,%d) | (%d,%d] | %d | %s | %s | %s | %s |" %
                  (m0, m1, r0, r1, cnt, fmt(top[0]), fmt(top[1]), fmt(top[2]), fmt(worst)))
    with open(os.path.join(args.out_dir, "autotune_batch_classes.md"), "w") as f:
        f.write("\n".join(md) + "\n")
    log("wrote", os.path.join(args.out_dir, "tuned_table.inc"))


if __name__ == "__main__":
    main()
