"""GPU parity on unstructured meshes: Delaunay triangulations of seeded random
points in the unit square / cube (scipy.spatial.Delaunay), relabelled with
shuffled local vertex orders.

Unlike the structured cases, these have irregular valences (rows of many
lengths, uneven tile element lists) and badly shaped elements (the smallest
|det B_K| is a few hundredths of a percent of the median in 3D). The bars are
the same as on the structured meshes: topology and CSR pattern bit-exact
against the oracle, values within relative Frobenius 1e-12, bitwise symmetric
and deterministic; the adjoint of L = u^T (K(a) + M(b)) u within 1e-12 of the
oracle's gradient (relative to its largest entry), both entry points; a
batch of mixed Delaunay meshes bitwise equal to single-mesh launches.
"""
import numpy as np
import pytest

import oracle
from gpu_util import dev_tensors, relabel, say
from oracle.gradient import grad_coefficients, grad_nodes, positions, quadratic_weights
from test_gpu_parity import check_against_oracle, run_case

pytestmark = pytest.mark.gpu

GTOL = 1e-12


def delaunay_mesh(dim, n_points, seed):
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(seed)
    corners = np.array(np.meshgrid(*[[0.0, 1.0]] * dim, indexing="ij")).reshape(dim, -1).T
    pts = np.concatenate([corners, rng.random((n_points, dim))])
    elems = Delaunay(pts).simplices.astype(np.int32)
    # drop elements that are flat to rounding (none are expected for random
    # points, but the hull can produce them)
    x = pts[elems]
    B = np.stack([x[:, q + 1] - x[:, 0] for q in range(dim)], axis=2)
    J = np.linalg.det(B)
    elems = elems[np.abs(J) > 1e-12 * np.abs(J).max()]
    used = np.unique(elems)
    remap = -np.ones(pts.shape[0], dtype=np.int64)
    remap[used] = np.arange(used.size)
    nodes, elems = relabel(pts[used], remap[elems].astype(np.int32), seed + 100)
    a = rng.lognormal(0, 0.5, elems.shape[0])
    b = rng.uniform(0.5, 2.0, elems.shape[0])
    return nodes, elems, a, b, rng


CASES = [(2, 3000, 1, "ned"), (2, 3000, 1, "rt"), (3, 2500, 2, "ned"), (3, 2500, 2, "rt"),
         (3, 400, 3, "ned")]


@pytest.mark.parametrize("dim,n_points,seed,kind", CASES,
                         ids=[f"{c[0]}d-{c[1]}pts-seed{c[2]}-{c[3]}" for c in CASES])
def test_forward_on_delaunay_meshes(dim, n_points, seed, kind):
    nodes, elems, a, b, _ = delaunay_mesh(dim, n_points, seed)
    g = run_case(f"delaunay {dim}D {n_points} points", nodes, elems, kind, a, b)
    check_against_oracle(g, nodes, elems, kind, a, b)


@pytest.mark.parametrize("dim,kind", [(2, "ned"), (3, "ned"), (3, "rt")])
def test_adjoint_on_delaunay_meshes(dim, kind):
    import torch
    import paper_1409_4618_amd as fem
    nodes, elems, a, b, rng = delaunay_mesh(dim, 300 if dim == 3 else 400, 7)
    say(f"[gpu] adjoint on a Delaunay mesh: {dim}D {kind} T={elems.shape[0]}")
    csr, topo = oracle.assemble(nodes, elems, kind, a=a, b=b)
    u = rng.normal(size=csr.n_rows)
    w = quadratic_weights(csr, u)
    pos = positions(csr, oracle.element_dofs(topo, kind))
    ga_o, gb_o = grad_coefficients(nodes, elems, kind, topo, pos, w, w)
    gn_o = grad_nodes(nodes, elems, kind, topo, pos, w, w, a, b)
    tn, te, ta, tb = dev_tensors(nodes, elems, a, b)
    mesh = fem.Mesh(tn, te)
    rowptr, colind = mesh.pattern(kind)
    tu = torch.tensor(u, device=tn.device)
    rows = torch.repeat_interleave(torch.arange(rowptr.numel() - 1, device=tn.device), torch.diff(rowptr))
    tw = tu[rows] * tu[colind.long()]
    gn, ga, gb = fem.assemble_backward(mesh, kind, tn, ta, tb, tw, tw)
    qn, qa, qb = fem.assemble_backward_quadratic(mesh, kind, tn, ta, tb, tu)
    mesh.status()
    for got, ref, nm in ((ga, ga_o, "a"), (gb, gb_o, "b"), (gn, gn_o, "x"),
                         (qa, ga_o, "a (quadratic)"), (qb, gb_o, "b (quadratic)"), (qn, gn_o, "x (quadratic)")):
        got = got.cpu().numpy()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        say(f"    dL/d{nm}: max rel err {err:.2e}")
        assert err <= GTOL, (nm, err)


@pytest.mark.parametrize("rows", [0, 128])
def test_batch_of_delaunay_meshes(rows):
    """Mixed 2D/3D Delaunay meshes of both kinds in one batched launch (and its
    graph replay): bitwise equal to single-mesh launches."""
    import torch
    import paper_1409_4618_amd as fem
    specs = [(2, 500, 11, "ned"), (3, 300, 12, "rt"), (3, 700, 13, "ned"), (2, 1500, 14, "rt"),
             (3, 150, 15, "ned"), (2, 90, 16, "ned")]
    say(f"[gpu] batch of {len(specs)} Delaunay meshes, rows_per_tile={rows}")
    meshes, kinds, nodes, a, b, Ks, Ms, refs = [], [], [], [], [], [], [], []
    for dim, n, seed, kind in specs:
        nd, el, ca, cb, _ = delaunay_mesh(dim, n, seed)
        tn, te, ta, tb = dev_tensors(nd, el, ca, cb)
        m = fem.Mesh(tn, te)
        K, M = fem.assemble(m, kind, tn, ta, tb)
        meshes.append(m)
        kinds.append(kind)
        nodes.append(tn)
        a.append(ta)
        b.append(tb)
        refs.append((K, M))
        Ks.append(torch.full_like(K, float("nan")))
        Ms.append(torch.full_like(M, float("nan")))
    B = fem.Batch(meshes, kinds)
    B.bind(nodes, a, b, Ks, Ms)
    B.set_config(rows, 1)
    B.assemble()
    torch.cuda.synchronize()
    for i, ((K, M), (Kr, Mr)) in enumerate(zip(zip(Ks, Ms), refs)):
        assert torch.equal(K, Kr) and torch.equal(M, Mr), i
    for K, M in zip(Ks, Ms):
        K.zero_()
        M.zero_()
    B.graph_launch()
    torch.cuda.synchronize()
    for i, ((K, M), (Kr, Mr)) in enumerate(zip(zip(Ks, Ms), refs)):
        assert torch.equal(K, Kr) and torch.equal(M, Mr), i
    for m in meshes:
        m.status()


def test_sweep_of_random_delaunay_meshes():
    """24 seeded meshes of random size (8 to 1500 points, both dimensions and
    kinds): each against the oracle, to the same bars, in one process."""
    rng = np.random.default_rng(2024)
    for i in range(24):
        dim = 2 + (i % 2)
        kind = "ned" if (i // 2) % 2 == 0 else "rt"
        n_points = int(rng.integers(8, 1500 if dim == 2 else 600))
        nodes, elems, a, b, _ = delaunay_mesh(dim, n_points, 1000 + i)
        g = run_case(f"sweep {i}: delaunay {dim}D {n_points} points", nodes, elems, kind, a, b)
        check_against_oracle(g, nodes, elems, kind, a, b)
