"""Build the HIP library libmlg.so in-tree for gfx950 with hipcc.

Every source is compiled to an object of its own (in parallel, under _build/ at the repository
root), then the objects are linked into one shared library.  Run as
``python -m paper_2609_18026_amd.build``; ``__graft_entry__.build()`` calls ``build()``.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmlg.so")
OBJDIR = os.path.join(os.path.dirname(HERE), "_build")
SOURCES = ["plan.cpp", "api.cpp", "kernels.hip", "fft256.hip", "gemm_fused.hip", "gemm_fold.hip", "gemm_split.hip",
           "batch.hip", "step.hip", "closure.hip", "symeig.cpp", "poisson.hip"]

# -packed-fp32-ops is a device target feature (the host pass warns that it does not know it)
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _jobs() -> int:
    n = os.cpu_count() or 4
    return max(1, min(n, 16, len(SOURCES)))


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        res = subprocess.run(cmd, capture_output=True, text=True)
        return src, obj, cmd, res

    with ThreadPoolExecutor(_jobs()) as ex:
        results = list(ex.map(compile_one, SOURCES))
    failed = [r for r in results if r[3].returncode != 0]
    for src, _, cmd, res in results:
        if verbose:
            print(" ".join(cmd), flush=True)
    if failed:
        for src, _, cmd, res in failed:
            sys.stderr.write(f"--- {src}\n" + res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libmlg.so: " + ", ".join(r[0] for r in failed))
    tmp = LIB + ".tmp"
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *[r[1] for r in results], "-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    res = subprocess.run(link, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("linking libmlg.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
