"""The checked build (libfem_check.so, selected with FEM_CHECK=1) on the GPU.

Its kernels compare every map index they read through with the size of what it
indexes and flag a violation through the mesh's status instead of touching
memory out of range. tests/checked_workload.py runs a fixed workload over every
kernel family (forward on both paths, batch tilings, adjoints, quadratic form,
integration, CG, P1 and majorant pieces) in a child process with the checked
build, and once in this process with the production build: the checked run
must find no index out of range (a flagged check raises there), and its results
must be bitwise those of the production build (the checks change no
arithmetic).
"""
import os
import subprocess
import sys

import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHECK_LIB = os.path.join(ROOT, "paper_1409_4618_amd", "libfem_check.so")


@pytest.mark.parametrize("env", [{}, {"FEM_FWD_PATH": "rows"}], ids=["ema", "rows"])
def test_checked_build_finds_nothing_and_matches(tmp_path, env):
    import checked_workload
    if not os.path.exists(CHECK_LIB):
        pytest.fail("libfem_check.so is missing: build it with __graft_entry__.build()")
    say(f"[gpu] checked build, workload in a child process {env}")
    child = tmp_path / "checked"
    child.mkdir()
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "checked_workload.py"), ROOT, str(child)],
                       capture_output=True, text=True, timeout=240,
                       env={**os.environ, "FEM_CHECK": "1", **env})
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-3000:]
    assert "checked workload done" in r.stdout
    say("[gpu] production build, same workload in this process")
    ref = checked_workload.run(str(tmp_path))
    got = np.load(child / "results.npz")
    assert sorted(got.files) == sorted(ref)
    for k in sorted(ref):
        assert np.array_equal(got[k], ref[k], equal_nan=False), k
    say(f"    {len(ref)} result arrays bitwise equal")
