"""The forward paths that an environment variable selects once per process,
each in a child process, against the oracle: FEM_EMA_THREADS=128 (element-major
tiles of 128 lanes) and FEM_FWD_PATH=rows (the row kernels for every mesh).
Same bars as the default path: pattern bit-exact, values within relative
Frobenius 1e-12, deterministic."""
import os
import subprocess
import sys

import numpy as np
import pytest

import meshgen as mg
import oracle
from gpu_util import TOL, rel_fro, relabel, say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CASES = [
    ("kuhn765", lambda: relabel(*mg.kuhn_box(7, 6, 5), 2), "ned"),
    ("kuhn765", lambda: relabel(*mg.kuhn_box(7, 6, 5), 2), "rt"),
    ("square97", lambda: relabel(*mg.unit_square(9, 7), 1), "ned"),
    ("kuhn12", lambda: mg.kuhn_box(12), "ned"),
]

CHILD = r"""
import sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
import paper_1409_4618_amd as fem
d = sys.argv[2]
for tag in sys.argv[3:]:
    z = np.load(f"{d}/{tag}.npz")
    kind = str(z["kind"])
    dev = torch.device("cuda:0")
    tn = torch.tensor(z["nodes"], device=dev)
    te = torch.tensor(z["elems"], device=dev)
    ta = torch.tensor(z["a"], device=dev)
    tb = torch.tensor(z["b"], device=dev)
    m = fem.Mesh(tn, te)
    K, M = fem.assemble(m, kind, tn, ta, tb)
    K2, M2 = fem.assemble(m, kind, tn, ta, tb)
    m.status()
    rowptr, colind = m.pattern(kind)
    np.savez(f"{d}/{tag}_out.npz", K=K.cpu().numpy(), M=M.cpu().numpy(), K2=K2.cpu().numpy(),
             M2=M2.cpu().numpy(), rowptr=rowptr.cpu().numpy(), colind=colind.cpu().numpy())
    print("done", tag, flush=True)
"""


@pytest.mark.parametrize("env", [{"FEM_EMA_THREADS": "128"}, {"FEM_FWD_PATH": "rows"}],
                         ids=["ema128", "rows"])
def test_selected_forward_path_matches_oracle(tmp_path, env):
    say(f"[gpu] forward path {env} in a child process")
    tags, refs = [], {}
    for i, (name, maker, kind) in enumerate(CASES):
        nodes, elems = maker()
        rng = np.random.default_rng(40 + i)
        nodes = mg.perturb_interior(np.asarray(nodes, dtype=np.float64), 0.05, 0.2, rng)
        a = rng.lognormal(0, 0.5, elems.shape[0])
        b = rng.uniform(0.5, 2.0, elems.shape[0])
        tag = f"{name}_{kind}"
        np.savez(tmp_path / f"{tag}.npz", nodes=nodes, elems=np.asarray(elems, np.int32), a=a, b=b, kind=kind)
        tags.append(tag)
        refs[tag] = oracle.assemble(nodes, elems, kind, a=a, b=b)[0]
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, str(tmp_path), *tags], capture_output=True,
                       text=True, timeout=180, env={**os.environ, **env})
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-3000:]
    for tag in tags:
        g = np.load(tmp_path / f"{tag}_out.npz")
        csr = refs[tag]
        assert np.array_equal(g["rowptr"], csr.rowptr) and np.array_equal(g["colind"], csr.colind), tag
        eK, eM = rel_fro(g["K"], csr.Kv), rel_fro(g["M"], csr.Mv)
        say(f"    {tag}: rel err K={eK:.2e} M={eM:.2e}")
        assert eK <= TOL and eM <= TOL, tag
        assert np.array_equal(g["K"], g["K2"]) and np.array_equal(g["M"], g["M2"]), tag
