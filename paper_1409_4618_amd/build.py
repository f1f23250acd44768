"""Build libfem.so (HIP, gfx950) in-tree, and its checked twin.

    python -m paper_1409_4618_amd.build        # or __graft_entry__.build()

Each source is compiled to an object under ``_build/`` in parallel with hipcc,
then linked into ``paper_1409_4618_amd/libfem.so``. The same sources built
with ``-DFEM_CHECK=1`` (objects under ``_build/check/``) give
``paper_1409_4618_amd/libfem_check.so``: every kernel compares the map indices
it reads through with the sizes of what they index and reports a violation
through the mesh's status instead of touching memory out of range. The
binding loads it instead of libfem.so when the environment has FEM_CHECK=1.
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
LIB_CHECK = os.path.join(HERE, "libfem_check.so")
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


def _compile(job) -> str:
    src, check = job
    out_dir = os.path.join(BUILD, "check") if check else BUILD
    obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, *DEVICE_FLAGS, *SOURCE_FLAGS.get(src, []), *(["-DFEM_CHECK=1"] if check else []),
           "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def _link(objs, lib):
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)


def build(verbose: bool = False, check: bool = True) -> str:
    """Compile libfem.so and, unless check is False, libfem_check.so."""
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(os.path.join(BUILD, "check"), exist_ok=True)
    jobs = [(src, False) for src in SOURCES] + ([(src, True) for src in SOURCES] if check else [])
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, jobs))
    _link(objs[:len(SOURCES)], LIB)
    if verbose:
        print("built", LIB)
    if check:
        _link(objs[len(SOURCES):], LIB_CHECK)
        if verbose:
            print("built", LIB_CHECK)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
