"""Build libbidiag.so in-tree with hipcc for gfx950.

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
SOURCES = ["kernels.hip", "adjoint.hip", "api.cpp", "plan.cpp", "adjoint_ops.cpp"]
ARCH = "gfx950"


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile every source (always) and link paper_1611_06892_amd/libbidiag.so."""
    hipcc = _hipcc()
    os.makedirs(OBJDIR, exist_ok=True)
    common = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-I", os.path.join(HERE, "..", "include")]
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(OBJDIR, src + ".o")
        if src.endswith(".hip"):
            cmd = [hipcc, "-x", "hip", "--offload-arch=" + ARCH, "-munsafe-fp-atomics",
                   "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                   *common, "-c", path, "-o", obj]
        else:
            cmd = [hipcc, *common, "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd, stderr=None if verbose else subprocess.DEVNULL
                              if False else None)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    link = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
