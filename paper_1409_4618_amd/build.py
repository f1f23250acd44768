"""Build libfem.so (HIP, gfx950) in-tree.

    python -m paper_1409_4618_amd.build        # or __graft_entry__.build()

Each source is compiled to an object under ``_build/`` in parallel with hipcc,
then linked into ``paper_1409_4618_amd/libfem.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libfem.so")
SOURCES = ["radix_sort.hip", "topology.hip", "assemble.hip", "adjoint.hip", "solve.hip", "integrate.hip", "p1.hip", "noalloc.hip", "api.hip"]
ARCH = os.environ.get("FEM_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
# Packed FP32 instructions are disabled for all device code (the path is FP64;
# this keeps the compiler from emitting v_pk_*_f32 anywhere).
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall",
          "-Wno-unused-function", "-Wno-unused-variable", "-I", os.path.join(ROOT, "include")]


# Per-source flags. The assembly kernels are built without floating-point
# contraction: every product is rounded on its own, so the same element entry
# gets bitwise the same value in whichever unrolled copy of the slot loop it
# is computed (this keeps K and M bitwise symmetric and deterministic). The
# adjoint (adjoint.hip) has no such constraint and keeps hipcc's default
# contraction into FMAs.
SOURCE_FLAGS = {"assemble.hip": ["-ffp-contract=off"]}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, *DEVICE_FLAGS, *SOURCE_FLAGS.get(src, []), "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
