"""Build ``libparem.so`` (HIP for gfx950) in-tree with hipcc.

Run as ``python -m paper_1412_1741_amd.build``. Every call compiles: each
source becomes an object under ``_build/`` (in parallel), then one link.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libparem.so")

SOURCES = [
    "parem_api.cpp",
    "parem_regex.cpp",
    "parem_walk.hip",
    "parem_walk_kgram_all.hip",
    "parem_walk_kgram_sel.hip",
    "parem_walk_kgram_redo.hip",
    "parem_walk_bytelds_all.hip",
    "parem_walk_bytelds_sel.hip",
    "parem_walk_bytelds_redo.hip",
    "parem_walk_byteglobal_all.hip",
    "parem_walk_byteglobal_sel.hip",
    "parem_walk_byteglobal_redo.hip",
    "parem_walk_hot_all.hip",
    "parem_walk_hot_sel.hip",
    "parem_walk_hot_redo.hip",
    "parem_walk_class_all.hip",
    "parem_walk_class_sel.hip",
    "parem_walk_class_redo.hip",
    "parem_walk_sparse_all.hip",
    "parem_walk_sparse_sel.hip",
    "parem_walk_sparse_redo.hip",
    "parem_mlp.hip",
    "parem_positions.hip",
    "parem_noalloc.hip",
    "parem_measure.hip",
    "parem_batch.hip",
    "parem_batch_t64.hip",
    "parem_batch_t128.hip",
    "parem_batch_t64_sel.hip",
    "parem_batch_t128_sel.hip",
]

HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # packed FP32 instructions are kept out of every HIP build
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def _jobs() -> int:
    for var in ("MAX_JOBS", "CMAKE_BUILD_PARALLEL_LEVEL"):
        v = os.environ.get(var)
        if v and v.isdigit() and int(v) > 0:
            return min(int(v), 16)
    return max(1, min(os.cpu_count() or 1, 16))


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [hipcc(), *HIP_FLAGS, "-I", os.path.join(HERE, "..", "include"), "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed compiling {os.path.basename(src)}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    with cf.ThreadPoolExecutor(max_workers=_jobs()) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    # -z defs: every symbol the units use must be defined by them or a linked library
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,-z,defs", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking libparem.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
