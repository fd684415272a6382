"""Build libbidiag.so in-tree with hipcc for gfx950.

The tile kernels are compiled once per (tile size, kernel family) pair (nb =
32, 64, 128, 256; reductions with FP64, FP32 or split-FP32 updates, and the
applications of Q and P) and once for their size-independent part, from the
same source, in parallel with the adjoint, the band-to-singular-value
kernels and the host sources.

Usage: python -m paper_1611_06892_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbidiag.so")
OBJDIR = os.path.join(HERE, "_build")
ARCH = "gfx950"
TILE_SIZES = (32, 64, 128, 256)
PRECS = (0, 2, 3)
HOST_SOURCES = ["api.cpp", "plan.cpp", "adjoint_ops.cpp"]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _jobs():
    """(object, command) for every translation unit."""
    hipcc = _hipcc()
    common = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-I", os.path.join(HERE, "..", "include")]
    device = [hipcc, "-x", "hip", "--offload-arch=" + ARCH, "-munsafe-fp-atomics", "-Wno-unneeded-internal-declaration",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *common]
    jobs = []
    kern = os.path.join(CSRC, "kernels.hip")
    for nb in (0,) + TILE_SIZES:        # 0: the kernels of batches mixing tile sizes 32 .. 128
        for prec in PRECS + ((1,) if nb else ()):       # 1: the application kernels
            obj = os.path.join(OBJDIR, "kernels_nb%d_p%d.o" % (nb, prec))
            jobs.append((obj, [*device, "-DBB_KERNELS_NB=%d" % nb, "-DBB_KERNELS_PREC=%d" % prec,
                               "-c", kern, "-o", obj]))
    obj = os.path.join(OBJDIR, "kernels_common.o")
    jobs.append((obj, [*device, "-DBB_KERNELS_COMMON", "-c", kern, "-o", obj]))
    for src in ("adjoint.hip", "ge2val.hip"):
        obj = os.path.join(OBJDIR, src.replace(".hip", ".o"))
        jobs.append((obj, [*device, "-c", os.path.join(CSRC, src), "-o", obj]))
    for src in HOST_SOURCES:
        obj = os.path.join(OBJDIR, src + ".o")
        jobs.append((obj, [hipcc, *common, "-c", os.path.join(CSRC, src), "-o", obj]))
    return hipcc, jobs


def build(verbose: bool = False, parallel: int = 0) -> str:
    """Compile every source (always) and link paper_1611_06892_amd/libbidiag.so."""
    hipcc, jobs = _jobs()
    os.makedirs(OBJDIR, exist_ok=True)
    width = parallel or max(1, min(len(jobs), os.cpu_count() or 1))
    pending = list(jobs)
    running = []
    failed = []
    # the slowest translation units (the largest tile sizes) start first
    pending.sort(key=lambda j: 0 if "kernels_nb256" in j[0] else 1 if "kernels_nb128" in j[0] else 2)
    while pending or running:
        while pending and len(running) < width:
            obj, cmd = pending.pop(0)
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((obj, cmd, subprocess.Popen(cmd)))
        obj, cmd, proc = running.pop(0)
        if proc.wait() != 0:
            failed.append(" ".join(cmd))
    if failed:
        raise RuntimeError("compilation failed:\n" + "\n".join(failed))
    tmp = LIB + ".tmp%d" % os.getpid()
    link = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *[o for o, _ in jobs]]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
