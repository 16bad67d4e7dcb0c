"""Builds the HIP library libsph_mi355x.so in-tree for gfx950 (hipcc).

A second build, libsph_mi355x_count.so (``--count``), defines SPH_COUNT_WALK:
the same kernels with tallies of the candidates their walks test and the
list entries they keep, read by ``profile_pass --walk-counts``; not for
production runs (one atomic per walk call)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsph_mi355x.so")
BUILD = os.path.join(HERE, "_build")
COUNT_LIB = os.path.join(HERE, "libsph_mi355x_count.so")
COUNT_BUILD = os.path.join(HERE, "_build_count")
SOURCES = ["build.hip", "tree.hip", "passes.hip", "passes_shared.hip", "adjoint.hip", "step.hip", "api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # packed FP32 instructions are kept out of generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable",
]


def _compile(src: str, count: bool = False) -> str:
    obj = os.path.join(COUNT_BUILD if count else BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + (["-DSPH_COUNT_WALK"] if count else [])
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, count: bool = False) -> str:
    lib = COUNT_LIB if count else LIB
    os.makedirs(COUNT_BUILD if count else BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda src: _compile(src, count), SOURCES))
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    import sys
    build(verbose=True, count="--count" in sys.argv[1:])
