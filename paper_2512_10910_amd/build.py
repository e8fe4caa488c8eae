"""Build libpne.so (HIP for gfx950 + host C++17) in-tree with hipcc."""

from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libpne.so")
SOURCES = ["bp.hip", "bp_persistent.hip", "kernels.hip", "strips.hip", "rankr.hip", "runtime.cpp", "geometry.cpp", "server.cpp", "noalloc.hip", "rankr_large.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-pthread",
    # packed FP32 arithmetic stays off (scalar FP32 code only)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-I", CSRC,
]
OBJDIR = os.path.join(PKG, "_build")


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel) and link libpne.so; always rebuilds."""
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(OBJDIR, exist_ok=True)
    tag = f"{os.getpid()}"
    objs = [os.path.join(OBJDIR, os.path.splitext(s)[0] + f".{tag}.o") for s in SOURCES]

    def compile_one(i):
        cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, SOURCES[i]), "-o", objs[i]]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)

    workers = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8"))))
    try:
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(compile_one, range(len(SOURCES))))
        tmp = LIB + f".tmp{tag}"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
