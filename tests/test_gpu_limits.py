"""The index limit at its edge, on a mesh larger than any benchmark: Kuhn 216^3
(60,466,176 tets, 10,218,313 nodes).

* Topology still fits (6 edge slots per tet: 363 M < 2^31) and its counts equal
  the Kuhn closed forms (E = 3n(n+1)^2 + 3n^2(n+1) + n^3, F = 1 - V + E + T by
  Euler's formula).
* The numbering at this size, where V > 2,642,245 makes the face keys take
  their edge-id form: edge and face rows are sorted node tuples in strictly
  increasing lexicographic order (so unique), every sampled element's local
  edges and faces are the rows its element map names, and its sign data equal
  the oracle's per-element sign rules.
* The Nedelec pattern would have n_elems * 36 = 2,176,782,336 >= 2^31 element
  pairs: fem_pattern refuses it with FEM_EOVERFLOW (status 5) before
  allocating, and the handle stays usable.
"""
import numpy as np
import pytest

import meshgen as mg
import oracle
from oracle.reference import LOCAL_EDGES, LOCAL_FACES
from gpu_util import say

pytestmark = pytest.mark.gpu


def test_pattern_beyond_the_index_limit_is_refused():
    import torch
    import paper_1409_4618_amd as fem
    from paper_1409_4618_amd import FemError
    n = 216
    nodes, elems = mg.kuhn_box(n)
    T = elems.shape[0]
    assert T * 36 >= 2 ** 31 > T * 6
    say(f"[gpu] index limit: Kuhn {n}^3, T={T}")
    d = torch.device("cuda:0")
    tn = torch.tensor(nodes, device=d)
    te = torch.tensor(elems, device=d)
    del nodes, elems
    mesh = fem.Mesh(tn, te)
    V, T_, E, F = mg.kuhn_counts(n)
    assert (mesh.n_nodes, mesh.n_elems, mesh.n_edges, mesh.n_faces) == (V, T_, E, F)
    assert V > 2_642_245
    say("    numbering properties")
    check_numbering(mesh, te)
    with pytest.raises(FemError) as ei:
        mesh.pattern_info("ned")
    assert ei.value.status == 5
    mesh.status()
    # a second request is refused the same way
    with pytest.raises(FemError) as ei:
        mesh.pattern_info("ned")
    assert ei.value.status == 5


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
