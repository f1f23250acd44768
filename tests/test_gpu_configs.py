"""Parity at the full benchmark sizes, in the launch configuration bench.py times.

* topology (edge / face numbering, element maps, sign data): bit-exact against
  the oracle's full numbering;
* CSR pattern and values: the whole matrices against the oracle's full
  assembly, element by element, for the 2D 32x32 square and Kuhn 64^3 (the
  oracle takes about half a minute on the latter); for the 96^3 and 128^3
  meshes every row of a sample (first and last tiles, random rows) against the
  oracle's row-wise assembly. Pattern bit-exact, values within relative
  Frobenius 1e-12;
* size-independent identities on the whole GPU output: nnz formula, bitwise
  symmetry, determinism, K G = 0 (Nedelec) and the constant-field identity
  u^T M(b) u = |c|^2 sum_K b_K |K|.
"""
import numpy as np
import pytest

import meshgen as mg
import oracle
from gpu_util import TOL, dev_tensors, rel_fro, say

pytestmark = pytest.mark.gpu

CONFIGS = {
    "square32_ned2d": mg.square_ned32,
    "kuhn64_ned3d": mg.kuhn64_ned,
    "kuhn128_rt3d": mg.kuhn128_rt,
    "kuhn128_ned3d": mg.kuhn128_ned,
    "kuhn96_ned3d": mg.kuhn96_ned_grad,
}
# configurations compared with the oracle on every value
FULL = ("square32_ned2d", "kuhn64_ned3d")


def sample_rows(n_rows, rng, k=300):
    first = np.arange(min(n_rows, 64))
    last = np.arange(max(0, n_rows - 300), n_rows)
    rnd = rng.choice(n_rows, size=min(n_rows, k), replace=False)
    return np.unique(np.concatenate([first, last, rnd]))


@pytest.mark.parametrize("cfg", list(CONFIGS))
def test_full_size_config(cfg):
    import torch
    import paper_1409_4618_amd as fem
    p = CONFIGS[cfg]()
    kind = p.kind
    say(f"[gpu] {cfg}: T={p.T} V={p.nodes.shape[0]} kind={kind}")
    tn, te, ta, tb = dev_tensors(p.nodes, p.elems, p.a, p.b)
    mesh = fem.Mesh(tn, te)
    K, M = fem.assemble(mesh, kind, tn, ta, tb)
    K2, M2 = fem.assemble(mesh, kind, tn, ta, tb)
    mesh.status()
    assert torch.equal(K, K2) and torch.equal(M, M2)          # deterministic
    rowptr, colind = mesh.pattern(kind)
    N = rowptr.numel() - 1
    nnz = colind.numel()
    V, T = p.nodes.shape[0], p.T
    E, F = mesh.n_edges, mesh.n_faces

    # topology bit-exact against the oracle's full numbering
    say("    oracle topology")
    topo = oracle.build_topology(p.elems, V)
    tg = mesh.topology()
    assert np.array_equal(tg["edges2nodes"].cpu().numpy(), topo.edges2nodes)
    assert np.array_equal(tg["elems2edges"].cpu().numpy(), topo.elems2edges)
    assert np.array_equal(tg["signs_e"].cpu().numpy(), topo.signs_e)
    if p.dim == 3:
        assert np.array_equal(tg["faces2nodes"].cpu().numpy(), topo.faces2nodes)
        assert np.array_equal(tg["elems2faces"].cpu().numpy(), topo.elems2faces)
        assert np.array_equal(tg["signs_f"].cpu().numpy(), topo.signs_f)

    # nnz formulas (two dofs couple iff they share an element)
    if p.dim == 2:
        assert nnz == E + 6 * T
    elif kind == "ned":
        assert nnz == E + 6 * F + 6 * T
    else:
        assert nnz == F + 12 * T

    rng = np.random.default_rng(123)
    if cfg in FULL:
        # every value against the oracle's full assembly
        say("    oracle: full assembly")
        csr, _ = oracle.assemble(p.nodes, p.elems, kind, a=p.a, b=p.b, topo=topo)
        assert np.array_equal(rowptr.cpu().numpy(), csr.rowptr)
        assert np.array_equal(colind.cpu().numpy(), csr.colind)
        for got, ref, nm in ((K, csr.Kv, "K"), (M, csr.Mv, "M")):
            g = got.cpu().numpy()
            e_f = rel_fro(g, ref)
            e_max = np.abs(g - ref).max() / np.abs(ref).max()
            say(f"    full {nm}: rel Frobenius {e_f:.2e}, max entry error / max entry {e_max:.2e}")
            assert e_f <= TOL and e_max <= TOL
        del csr

    # sampled rows against the oracle's row-wise (dictionary) assembly
    rows = sample_rows(N, rng)
    say(f"    oracle rows: {rows.size}")
    ref, _ = oracle.assemble_rows(p.nodes, p.elems, kind, rows, a=p.a, b=p.b, topo=topo)
    rp = rowptr.cpu().numpy()
    sel = np.concatenate([np.arange(rp[r], rp[r + 1]) for r in rows])
    tsel = torch.tensor(sel, device=tn.device)
    cg = colind[tsel].cpu().numpy()
    kg = K[tsel].cpu().numpy()
    mg_ = M[tsel].cpu().numpy()
    co = np.concatenate([ref[r][0] for r in rows])
    ko = np.concatenate([ref[r][1] for r in rows])
    mo = np.concatenate([ref[r][2] for r in rows])
    assert np.array_equal(cg, co)
    eK, eM = rel_fro(kg, ko), rel_fro(mg_, mo)
    say(f"    sampled rows rel err K={eK:.2e} M={eM:.2e}")
    assert eK <= TOL and eM <= TOL

    # bitwise symmetry of the whole matrices
    rows_t = torch.repeat_interleave(torch.arange(N, device=tn.device), torch.diff(rowptr))
    keys = rows_t * N + colind.long()
    tkeys = colind.long() * N + rows_t
    pos = torch.searchsorted(keys, tkeys)
    assert torch.equal(keys[pos], tkeys)
    assert torch.equal(K[pos], K) and torch.equal(M[pos], M)
    del keys, tkeys, pos

    # constant-field identity and K G = 0 on the whole output
    c = torch.tensor(rng.normal(size=p.dim), device=tn.device)
    X = torch.tensor(p.nodes, device=tn.device)
    if kind == "ned" or p.dim == 2:
        e2n = tg["edges2nodes"].long()
        u = ((X[e2n[:, 0]] - X[e2n[:, 1]]) * c).sum(dim=1)
    else:
        f2n = tg["faces2nodes"].long()
        # elementwise (an (N,3) @ (3,) product is not used: the library gemv
        # returns wrong values for N > 2^24 rows on this stack)
        u = (torch.linalg.cross(X[f2n[:, 1]] - X[f2n[:, 0]], X[f2n[:, 2]] - X[f2n[:, 0]]) * c).sum(dim=1)
    w = u[rows_t] * u[colind.long()]
    uMu = float((w * M).sum())
    uKu = float((w * K).sum())
    Xe = p.nodes[p.elems]
    Bm = np.transpose(Xe[:, 1:] - Xe[:, :1], (0, 2, 1))
    vol = np.abs(np.linalg.det(Bm)) / (2 if p.dim == 2 else 6)
    bb = np.ones(T) if p.b is None else p.b
    expect = float(np.sum(bb * vol) * np.dot(c.cpu().numpy(), c.cpu().numpy()))
    uKu_abs = float((w * K).abs().sum())
    say(f"    constant field: uMu rel err {abs(uMu - expect) / expect:.2e}, |uKu|/sum|wK| {abs(uKu) / uKu_abs:.2e}")
    assert abs(uMu - expect) <= 1e-12 * expect
    assert abs(uKu) <= 1e-12 * uKu_abs
    if kind == "ned":
        phi = torch.tensor(rng.normal(size=V), device=tn.device)
        e2n = tg["edges2nodes"].long()
        v = phi[e2n[:, 0]] - phi[e2n[:, 1]]
        y = torch.zeros(N, dtype=torch.float64, device=tn.device)
        y.index_add_(0, rows_t, K * v[colind.long()])
        rel = float(y.abs().max() / (K.abs().max() * v.abs().max()))
        say(f"    K G phi: max rel {rel:.2e}")
        assert rel <= 1e-12
