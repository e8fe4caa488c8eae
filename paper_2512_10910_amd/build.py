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


# The checked build (libpne_checked.so): the same library with the cluster
# kernels' index checks compiled in (PNE_CHECKED; a failed check suppresses
# the access and reports PNE_ERR_CHECK for the network).  Only the sources
# listed here differ from the plain build.
LIB_CHECKED = os.path.join(PKG, "libpne_checked.so")
CHECKED_SOURCES = ["kernels.hip"]


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel) and link libpne.so and
    libpne_checked.so; always rebuilds."""
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(OBJDIR, exist_ok=True)
    tag = f"{os.getpid()}"
    jobs = [(s, [], os.path.join(OBJDIR, os.path.splitext(s)[0] + f".{tag}.o")) for s in SOURCES]
    jobs += [(s, ["-DPNE_CHECKED=1"], os.path.join(OBJDIR, os.path.splitext(s)[0] + f".checked.{tag}.o"))
             for s in CHECKED_SOURCES]
    objs = [o for _, _, o in jobs]

    def compile_one(i):
        src, extra, obj = jobs[i]
        cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)

    def link(lib, lib_objs):
        tmp = lib + f".tmp{tag}"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", *lib_objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, lib)

    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", "8"))))
    try:
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(compile_one, range(len(jobs))))
        plain = objs[:len(SOURCES)]
        link(LIB, plain)
        checked = {s: o for s, _, o in jobs[len(SOURCES):]}
        link(LIB_CHECKED, [checked.get(s, o) for s, o in zip(SOURCES, plain)])
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
