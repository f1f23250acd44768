"""Register budgets of the hot kernels, read from the AMDGPU metadata of the
built libfem.so (CPU only: the code object is extracted from the library, no
GPU is touched).

Occupancy is what hides the gather latency of these memory-bound kernels, so
the budgets are part of the design: a VGPR count above a wavefront boundary
costs a wavefront per SIMD (gfx950: 512 VGPRs per lane per SIMD, allocated in
blocks of 8), and a spill (private segment) adds memory traffic. The batched
kernel over every kind holds every kind's tile body and sits exactly at its
boundary; the batch's per-kind grid kernels take their kind's registers (the
3D Nedelec one a few more than the single-mesh kernel: the mesh descriptor
comes from the table).
"""
import glob
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1409_4618_amd", "libfem.so")
LLVM = "/opt/rocm/llvm/bin"

# (mangled-name fragment, minimum wavefronts per SIMD)
BUDGETS = [
    ("k_forward_emaILi2ELi256", 6),   # 3D Nedelec forward
    ("k_forward_emaILi1ELi256", 8),   # 3D Raviart-Thomas forward
    ("k_forward_emaILi0ELi256", 8),   # 2D forward
    ("k_batch_emaILi256", 5),         # batched forward, all kinds
    ("k_batch_ema_gridILi2ELi256", 5),  # batched forward, one launch per kind: 3D Nedelec
    ("k_batch_ema_gridILi1ELi256", 8),  # 3D Raviart-Thomas
    ("k_batch_ema_gridILi0ELi256", 8),  # 2D
    ("k_backwardILi2ELi2", 4),        # 3D Nedelec adjoint, quadratic form
    ("k_backwardILi2ELi1", 3),        # 3D Nedelec adjoint, materialised weights
]


def kernel_metadata(tmp_path):
    if not os.path.exists(LIB):
        pytest.skip("libfem.so is not built")
    if not os.path.exists(os.path.join(LLVM, "llvm-objdump")):
        pytest.skip("ROCm llvm tools not available")
    lib = str(tmp_path / "libfem.so")
    shutil.copy(LIB, lib)
    subprocess.run([os.path.join(LLVM, "llvm-objdump"), "--offloading", lib], check=True,
                   capture_output=True, cwd=tmp_path, timeout=120)
    meta = {}
    for co in glob.glob(str(tmp_path / "libfem.so.*gfx950*")):
        notes = subprocess.run([os.path.join(LLVM, "llvm-readelf"), "--notes", co], check=True,
                               capture_output=True, text=True, timeout=120).stdout
        for block in notes.split("  - .agpr_count:")[1:]:
            name = re.search(r"\.name:\s+(\S+)", block)
            vgpr = re.search(r"\.vgpr_count:\s+(\d+)", block)
            agpr = re.search(r"^\s*(\d+)", block)
            priv = re.search(r"\.private_segment_fixed_size:\s+(\d+)", block)
            if name and vgpr and priv:
                meta[name.group(1)] = (int(vgpr.group(1)) + (int(agpr.group(1)) if agpr else 0),
                                       int(priv.group(1)))
    if not meta:
        pytest.skip("no gfx950 kernel metadata found")
    return meta


def waves_per_simd(vgprs):
    return 512 // max(8, (vgprs + 7) // 8 * 8)


def test_no_kernel_spills(tmp_path):
    meta = kernel_metadata(tmp_path)
    spills = {n: p for n, (_, p) in meta.items() if p}
    assert not spills, spills


@pytest.mark.parametrize("fragment,min_waves", BUDGETS)
def test_hot_kernel_occupancy(tmp_path, fragment, min_waves):
    meta = kernel_metadata(tmp_path)
    hits = {n: v for n, (v, _) in meta.items() if fragment in n}
    assert hits, fragment
    for name, vgprs in hits.items():
        assert waves_per_simd(vgprs) >= min_waves, (name, vgprs, waves_per_simd(vgprs))
