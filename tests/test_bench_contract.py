"""The benchmark's accounting, on the CPU (no GPU is touched).

* `bench.py --gpus N` with N > 1 refuses with a message: the library assembles on one
  GPU.
* The algorithmic bytes behind `roofline.achieved` equal the compulsory bytes
  written out independently from the Kuhn closed forms: a tet reads its four
  node ids (16 B) and two coefficients (16 B), every node's coordinates are
  read once (24 B), and K and M are written once (16 B per CSR entry), with
  nnz = E + 6F + 6T for Nedelec and F + 12T for Raviart-Thomas (adjacent edges
  couple through their faces, opposite edges through their tet; two faces
  couple through their one tet).
* The quadratic-form adjoint reads elems, coordinates, a, b and u (one value
  per edge) once and writes dL/da and dL/db.
"""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import meshgen as mg  # noqa: E402


def bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"] and line["n_gpus"] == 2


@pytest.mark.parametrize("n,kind,expected", [
    (64, "ned", 542_219_800),      # the headline: 344.7 B/tet
    (128, "ned", 4_324_736_024),   # the 128^3 target: 343.7 B/tet
    (128, "rt", 3_274_318_872),    # 260.2 B/tet
])
def test_forward_algorithmic_bytes(n, kind, expected):
    b = bench_module()
    V, T, E, F = mg.kuhn_counts(n)
    nnz = E + 6 * F + 6 * T if kind == "ned" else F + 12 * T
    by_hand = 16 * T + 16 * T + 24 * V + 16 * nnz
    assert by_hand == expected
    assert b.algorithmic_bytes(T, V, 3, nnz, True) == expected


def test_adjoint_algorithmic_bytes():
    b = bench_module()
    V, T, E, F = mg.kuhn_counts(96)
    assert T == 5_308_416
    by_hand = 16 * T + 24 * V + 16 * T + 8 * E + 16 * T
    assert by_hand == 326_919_192
    assert b.adjoint_bytes(T, V, 3, E) == by_hand
