"""The index limits at their edges, on meshes larger than any benchmark.

Kuhn 216^3 (60,466,176 tets, 10,218,313 nodes), 3D Nedelec:
* Topology fits (6 edge slots per tet: 363 M < 2^31) and its counts equal the
  Kuhn closed forms (E = 3n(n+1)^2 + 3n^2(n+1) + n^3, F = 1 - V + E + T by
  Euler's formula).
* The numbering at this size, where V > 2,642,245 makes the face keys take
  their edge-id form: edge and face rows are sorted node tuples in strictly
  increasing lexicographic order (so unique), every sampled element's local
  edges and faces are the rows its element map names, and its sign data equal
  the oracle's per-element sign rules.
* The pattern has 36 T = 2,176,782,336 >= 2^31 element pairs, sorted in
  chunks of whole rows: nnz = E + 6F + 6T, and the assembled K and M
  (1.16 G nonzeros each) are deterministic, bitwise symmetric, satisfy
  K G = 0 for the discrete gradient and the constant-field identity
  u^T M(b) u = |c|^2 sum_K b_K |K| on the whole output.

Kuhn 266^3 (112,926,576 tets): the Nedelec pattern would have more than
2^31 - 1 nonzeros (E + 6F + 6T = 2,167,610,858 at that size), so fem_pattern
refuses it with FEM_EOVERFLOW (status 5), keeps nothing of the attempt, and
the handle stays usable: the Raviart-Thomas pattern of the same mesh
(1.58 G nonzeros) still builds.
"""
import numpy as np
import pytest

import meshgen as mg
import oracle
from oracle.reference import LOCAL_EDGES, LOCAL_FACES
from gpu_util import say

pytestmark = pytest.mark.gpu


def kuhn_on_device(n):
    import torch
    nodes, elems = mg.kuhn_box(n)
    d = torch.device("cuda:0")
    return torch.tensor(nodes, device=d), torch.tensor(elems, device=d)


def test_kuhn216_beyond_2_31_element_pairs():
    import torch
    import paper_1409_4618_amd as fem
    n = 216
    tn, te = kuhn_on_device(n)
    T = te.shape[0]
    assert T * 36 >= 2 ** 31 > T * 6
    say(f"[gpu] index limit: Kuhn {n}^3, T={T}")
    mesh = fem.Mesh(tn, te)
    V, T_, E, F = mg.kuhn_counts(n)
    assert (mesh.n_nodes, mesh.n_elems, mesh.n_edges, mesh.n_faces) == (V, T_, E, F)
    assert V > 2_642_245
    say("    numbering properties")
    check_numbering(mesh, te)
    say("    pattern in row chunks")
    N, nnz = mesh.pattern_info("ned")
    assert N == E and nnz == E + 6 * F + 6 * T
    K, M = fem.assemble(mesh, "ned", tn)
    K2, M2 = fem.assemble(mesh, "ned", tn)
    mesh.status()
    assert torch.equal(K, K2) and torch.equal(M, M2)
    del K2, M2
    say("    whole-output identities")
    check_identities(mesh, tn, K, M)


def test_kuhn266_nedelec_pattern_is_refused():
    import paper_1409_4618_amd as fem
    from paper_1409_4618_amd import FemError
    n = 266
    tn, te = kuhn_on_device(n)
    V, T, E, F = mg.kuhn_counts(n)
    assert E + 6 * F + 6 * T >= 2 ** 31 > F + 12 * T
    say(f"[gpu] index limit: Kuhn {n}^3, T={T}")
    mesh = fem.Mesh(tn, te)
    with pytest.raises(FemError) as ei:
        mesh.pattern_info("ned")
    assert ei.value.status == 5
    mesh.status()
    N, nnz = mesh.pattern_info("rt")
    assert N == F and nnz == F + 12 * T


def check_identities(mesh, tn, K, M):
    """Bitwise symmetry, K G = 0 and the constant-field identity (b = 1) on
    the whole output (elementwise torch ops: no library gemv)."""
    import torch
    rowptr, colind = mesh.pattern("ned")
    N = rowptr.numel() - 1
    rows_t = torch.repeat_interleave(torch.arange(N, device=tn.device), torch.diff(rowptr))
    ci = colind.long()
    del colind
    keys = rows_t * N + ci
    pos = torch.searchsorted(keys, ci * N + rows_t)
    assert torch.equal(keys[pos], ci * N + rows_t)
    del keys
    assert torch.equal(K[pos], K) and torch.equal(M[pos], M)
    del pos
    t = mesh.topology()
    e2n = t["edges2nodes"].long()
    del t
    rng = np.random.default_rng(5)
    phi = torch.tensor(rng.normal(size=tn.shape[0]), device=tn.device)
    v = phi[e2n[:, 0]] - phi[e2n[:, 1]]
    y = torch.zeros(N, dtype=torch.float64, device=tn.device)
    y.index_add_(0, rows_t, K * v[ci])
    rel = float(y.abs().max() / (K.abs().max() * v.abs().max()))
    say(f"    K G phi: max rel {rel:.2e}")
    assert rel <= 1e-12
    del y, v, phi
    c = torch.tensor(rng.normal(size=3), device=tn.device)
    u = ((tn[e2n[:, 0]] - tn[e2n[:, 1]]) * c).sum(dim=1)
    w = u[rows_t] * u[ci]
    uMu = float((w * M).sum())
    uKu = float((w * K).sum())
    uKu_abs = float((w * K).abs().sum())
    expect = float((c * c).sum())  # sum of the element volumes of the unit cube, b = 1
    say(f"    constant field: uMu rel err {abs(uMu - expect) / expect:.2e}, |uKu|/sum|wK| {abs(uKu) / uKu_abs:.2e}")
    assert abs(uMu - expect) <= 1e-12 * expect
    assert abs(uKu) <= 1e-12 * uKu_abs


def strictly_increasing_rows(rows):
    """Consecutive rows of an int tensor [n, w] compare lexicographically greater."""
    import torch
    a, b = rows[:-1].long(), rows[1:].long()
    gt = torch.zeros(a.shape[0], dtype=torch.bool, device=rows.device)
    eq = torch.ones_like(gt)
    for c in range(rows.shape[1]):
        gt |= eq & (b[:, c] > a[:, c])
        eq &= b[:, c] == a[:, c]
    return bool(gt.all())


def check_numbering(mesh, te):
    import torch
    t = mesh.topology()
    e2n, f2n = t["edges2nodes"], t["faces2nodes"]
    assert bool((e2n[:, 0] < e2n[:, 1]).all()) and strictly_increasing_rows(e2n)
    assert bool((f2n[:, 0] < f2n[:, 1]).all()) and bool((f2n[:, 1] < f2n[:, 2]).all())
    assert strictly_increasing_rows(f2n)
    gen = torch.Generator(device=te.device)
    gen.manual_seed(7)
    s = torch.randint(0, te.shape[0], (1 << 20,), device=te.device, generator=gen)
    el = te[s].long()
    for k, (i, j) in enumerate(LOCAL_EDGES[3]):
        want = torch.stack([torch.minimum(el[:, i], el[:, j]), torch.maximum(el[:, i], el[:, j])], 1)
        assert torch.equal(e2n[t["elems2edges"][s, k].long()].long(), want), k
    for k, f in enumerate(LOCAL_FACES):
        want = torch.sort(el[:, list(f)], dim=1).values
        assert torch.equal(f2n[t["elems2faces"][s, k].long()].long(), want), k
    few = s[:4096]
    el_h = te[few].cpu().numpy()
    assert np.array_equal(t["signs_e"][few].cpu().numpy(), oracle.topology.signs_edges(el_h))
    assert np.array_equal(t["signs_f"][few].cpu().numpy(), oracle.topology.signs_faces(el_h))
    del t
    torch.cuda.empty_cache()
