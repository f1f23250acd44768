"""The index limit at its edge, on a mesh larger than any benchmark: Kuhn 216^3
(60,466,176 tets, 10,218,313 nodes).

* Topology still fits (6 edge slots per tet: 363 M < 2^31) and its counts equal
  the Kuhn closed forms (E = 3n(n+1)^2 + 3n^2(n+1) + n^3, F = 1 - V + E + T by
  Euler's formula).
* The Nedelec pattern would have n_elems * 36 = 2,176,782,336 >= 2^31 element
  pairs: fem_pattern refuses it with FEM_EOVERFLOW (status 5) before
  allocating, and the handle stays usable.
"""
import pytest

import meshgen as mg
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
    with pytest.raises(FemError) as ei:
        mesh.pattern_info("ned")
    assert ei.value.status == 5
    mesh.status()
    # a second request is refused the same way
    with pytest.raises(FemError) as ei:
        mesh.pattern_info("ned")
    assert ei.value.status == 5
