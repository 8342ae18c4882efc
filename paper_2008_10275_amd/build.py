"""Build the HIP library liblrcheb.so in-tree (gfx950).

Host-only factorisation code is compiled with g++ (OpenMP via libgomp, the
runtime torch also uses); kernels and the C ABI with hipcc for gfx950.
Run:  python -m paper_2008_10275_amd.build   (or __graft_entry__.build()).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "liblrcheb.so")

HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result"]
HOST_FLAGS = ["-O3", "-mavx2", "-mfma", "-fopenmp", "-fPIC", "-std=c++17"]

HIP_SOURCES = ["k_sparse.hip", "k_dense.hip", "k_small.hip", "k_mlp.hip", "solver.cpp", "batch.cpp",
               "tune.cpp", "capi.cpp", "prof.cpp", "noalloc.hip", "timedep.cpp", "gmrest.cpp"]
HOST_SOURCES = ["host/ndfact.cpp", "host/ilu0.cpp"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def _stale(src, obj, headers_mtime):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return t < os.path.getmtime(src) or t < headers_mtime


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (incremental=True: only objects older than their
    source or than any header) and link the library."""
    os.makedirs(BUILD, exist_ok=True)
    hdr = [os.path.join(r, f) for d in (CSRC, os.path.join(os.path.dirname(HERE), "include"))
           for r, _, fs in os.walk(d) for f in fs if f.endswith((".h", ".hpp"))]
    hmt = max(os.path.getmtime(h) for h in hdr)
    jobs = []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, os.path.basename(src).replace(".cpp", ".host.o"))
        jobs.append(["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        jobs.append(["hipcc", *HIP_FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj])
    todo = [j for j in jobs if not incremental or _stale(j[-3], j[-1], hmt)]
    with cf.ThreadPoolExecutor(max_workers=max(1, min(8, len(todo)))) as ex:
        for r in ex.map(_run, todo):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout + r.stderr, file=sys.stderr)
    objs = [j[-1] for j in jobs]
    tmp = LIB + ".tmp"
    _run(["hipcc", "--offload-arch=gfx950", "-shared", "-o", tmp, *objs, "-lgomp"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv))
