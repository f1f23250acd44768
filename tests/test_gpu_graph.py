"""fem_assemble captured into a HIP graph (torch.cuda.CUDAGraph) and replayed.

The single-mesh forward path launches one kernel and allocates nothing, so a
caller can capture it. Every replay must reproduce the eager launch bit for
bit, also after unrelated eager work (other assemblies, fills of the output
buffers) between the replays, for 2D and 3D, Nedelec and Raviart-Thomas.
"""
import numpy as np
import pytest

import meshgen as mg
from gpu_util import dev_tensors, say

pytestmark = pytest.mark.gpu


def _problem(dim, seed):
    rng = np.random.default_rng(seed)
    if dim == 2:
        nodes, elems = mg.unit_square(23, 19)
        h = 1 / 23
    else:
        nodes, elems = mg.kuhn_box(9, 8, 7)
        h = 1 / 9
    nodes = mg.perturb_interior(nodes, h, 0.2, rng)
    T = elems.shape[0]
    return nodes, elems, rng.lognormal(0, 0.5, T), rng.lognormal(0, 0.5, T)


@pytest.mark.parametrize("dim,kind", [(2, "ned"), (3, "ned"), (3, "rt"), (2, "rt")])
def test_captured_assembly_replays_bitwise(dim, kind):
    import torch
    import paper_1409_4618_amd as fem
    nodes, elems, a, b = _problem(dim, 11 + dim)
    say(f"[gpu] graph capture of fem_assemble, dim {dim}, {kind}, T={elems.shape[0]}")
    tn, te, ta, tb = dev_tensors(nodes, elems, a, b)
    mesh = fem.Mesh(tn, te)
    _, nnz = mesh.pattern_info(kind)
    K_ref = torch.empty(nnz, dtype=torch.float64, device=tn.device)
    M_ref = torch.empty_like(K_ref)
    fem.assemble_into(mesh, kind, tn, ta, tb, K_ref, M_ref)
    torch.cuda.synchronize()
    mesh.status()

    K = torch.empty_like(K_ref)
    M = torch.empty_like(K_ref)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fem.assemble_into(mesh, kind, tn, ta, tb, K, M)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fem.assemble_into(mesh, kind, tn, ta, tb, K, M)
    torch.cuda.synchronize()
    mesh.status()

    # eager work between the replays: the outputs overwritten, and an eager
    # assembly with other coefficients into other buffers
    K2 = torch.empty_like(K_ref)
    M2 = torch.empty_like(K_ref)
    for r in range(4):
        K.fill_(float("nan"))
        M.fill_(-1.0)
        fem.assemble_into(mesh, kind, tn, tb, ta, K2, M2)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        mesh.status()
        assert torch.equal(K, K_ref) and torch.equal(M, M_ref), f"replay {r}"
    # swapping a and b swaps the roles of the two matrices' coefficients only
    assert not torch.equal(K2, K_ref)
