"""Pins of the oracle's topology and sign data.

* brute force: a pure-Python set/dict numbering equals the vectorised one;
* Euler's formula V - E + T = 1 (2D disk) and V - E + F - T = 1 (3D ball);
* matrix sizes printed in the paper's Tables (3D cube, 2D L-shape, eddy square),
  from explicit meshes for the small levels;
* the sign rule of Section 3 on a single element, and the parity rule for 3D
  faces against the det-based orientation table of Section 2.3.
"""
import os

import numpy as np
import pytest

import meshgen as mg
from oracle.topology import (brute_force_topology, build_topology, signs_edges,
                             signs_faces, signs_faces_geometric)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_table_sizes.txt")


def load_sizes():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        t, lvl, p, col, v = line.split()
        rows.append((t, int(lvl), int(p), col, int(v)))
    return rows


def _relabel(nodes, elems, seed):
    """Random node relabelling and random local vertex order (mixed orientations)."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(nodes.shape[0])
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    nodes2 = nodes[perm]
    elems2 = inv[elems]
    for t in range(elems2.shape[0]):
        elems2[t] = elems2[t][rng.permutation(elems2.shape[1])]
    return nodes2, elems2.astype(np.int32)


@pytest.mark.parametrize("maker", [lambda: mg.unit_square(5, 4), lambda: mg.kuhn_box(3, 2, 2),
                                   lambda: mg.l_shape(3)])
def test_numbering_matches_brute_force(maker):
    nodes, elems = maker()
    for seed in (0, 1):
        n2, e2 = _relabel(nodes, elems, seed) if seed else (nodes, elems)
        topo = build_topology(e2, n2.shape[0])
        edges, el2e, faces, el2f = brute_force_topology(e2.tolist())
        assert topo.edges2nodes.tolist() == [list(e) for e in edges]
        assert topo.elems2edges.tolist() == el2e
        if topo.dim == 3:
            assert topo.faces2nodes.tolist() == [list(f) for f in faces]
            assert topo.elems2faces.tolist() == el2f


@pytest.mark.parametrize("m", [1, 2, 3, 8, 17])
def test_l_shape_torch_layout_equals_numpy(m):
    """The torch layout of the L-shape mesh (used for the large timing levels)
    is the numpy one: same node coordinates, same element lists."""
    import torch
    nodes, elems = mg.l_shape(m)
    tn, te = mg.l_shape_torch(m, "cpu")
    assert te.dtype == torch.int32 and tn.dtype == torch.float64
    assert np.array_equal(tn.numpy(), nodes) and np.array_equal(te.numpy(), elems)


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16])
def test_unit_square_torch_layout_equals_numpy(n):
    """The torch layout of the unit-square mesh (used for the large eddy-current
    meshes) is the numpy one: same node coordinates, same element lists."""
    import torch
    nodes, elems = mg.unit_square(n)
    tn, te = mg.unit_square_torch(n, "cpu")
    assert te.dtype == torch.int32 and tn.dtype == torch.float64
    assert np.array_equal(tn.numpy(), nodes) and np.array_equal(te.numpy(), elems)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_kuhn_box_torch_layout_equals_numpy(n):
    """The torch layout of the Kuhn cube mesh (used for the large timing
    levels) is the numpy one: same node coordinates, same element lists."""
    import torch
    nodes, elems = mg.kuhn_box(n)
    tn, te = mg.kuhn_box_torch(n, "cpu")
    assert te.dtype == torch.int32 and tn.dtype == torch.float64
    assert np.array_equal(tn.numpy(), nodes) and np.array_equal(te.numpy(), elems)


@pytest.mark.parametrize("n", [1, 2, 5, 9])
def test_euler_and_kuhn_closed_forms(n):
    nodes, elems = mg.kuhn_box(n)
    topo = build_topology(elems, nodes.shape[0])
    V, T, E, F = nodes.shape[0], elems.shape[0], topo.n_edges, topo.n_faces
    assert V - E + F - T == 1
    assert (V, T, E, F) == mg.kuhn_counts(n)
    nodes, elems = mg.unit_square(n, n + 1)
    topo = build_topology(elems, nodes.shape[0])
    assert nodes.shape[0] - topo.n_edges + elems.shape[0] == 1
    nodes, elems = mg.kuhn_box(n, n + 1, 2)
    topo = build_topology(elems, nodes.shape[0])
    assert nodes.shape[0] - topo.n_edges + topo.n_faces - elems.shape[0] == 1


def test_paper_table_sizes_explicit_meshes():
    checked = 0
    for table, lvl, p, col, val in load_sizes():
        if table == "3d" and p <= 24:
            nodes, elems = mg.kuhn_box(p)
            topo = build_topology(elems, nodes.shape[0])
            got = topo.n_faces if col == "faces" else topo.n_edges
        elif table == "2d" and p <= 128:
            nodes, elems = mg.l_shape(p)
            assert elems.shape[0] == 6 * 4 ** lvl
            got = build_topology(elems, nodes.shape[0]).n_edges
        elif table == "eddy" and p <= 512:
            nodes, elems = mg.unit_square(p)
            got = elems.shape[0] if col == "elems" else build_topology(elems, nodes.shape[0]).n_edges
        else:
            continue
        assert got == val, (table, lvl, col, got, val)
        checked += 1
    assert checked >= 12


def test_paper_table_sizes_closed_forms():
    """Larger levels: the closed forms behind the explicit-mesh counts above
    (Kuhn: E, F from kuhn_counts; L-shape: E = V + T - 1; square: E = 3n^2 + 2n)."""
    for table, lvl, p, col, val in load_sizes():
        if table == "3d":
            V, T, E, F = mg.kuhn_counts(p)
            assert (F if col == "faces" else E) == val
        elif table == "2d":
            V = (2 * p + 1) ** 2 - p * p
            T = 6 * p * p
            assert V + T - 1 == val
        else:
            assert (2 * p * p if col == "elems" else 3 * p * p + 2 * p) == val


def test_sign_rule_single_triangle():
    # Section 3: local edge 1 runs from node 2 to node 3 and gets +1 iff the global
    # index of node 2 exceeds that of node 3; edges 2, 3 follow cyclically.
    elems = np.array([[0, 1, 2], [2, 1, 0], [5, 9, 7]])
    s = signs_edges(elems)
    assert s.tolist() == [[-1, 1, -1], [1, -1, 1], [1, 1, -1]]


def test_sign_rule_single_tet():
    elems = np.array([[0, 1, 2, 3]])
    # Figure 1 arrows: 1->2, 1->3, 1->4, 2->3, 3->4, 4->2
    assert signs_edges(elems).tolist() == [[-1, -1, -1, -1, -1, 1]]
    assert signs_faces(elems).tolist() == [[-1, 1, -1, 1]]


def test_face_parity_rule_equals_det_table():
    nodes, elems = mg.kuhn_box(3, 3, 2)
    rng = np.random.default_rng(7)
    nodes = mg.perturb_interior(nodes, 1 / 3, 0.2, rng)
    nodes, elems = _relabel(nodes, elems, 11)
    topo = build_topology(elems, nodes.shape[0])
    X = nodes[elems]
    det = np.linalg.det(np.transpose(X[:, 1:] - X[:, :1], (0, 2, 1)))
    assert (det < 0).any() and (det > 0).any()
    geo = signs_faces_geometric(nodes, elems, topo.faces2nodes, topo.elems2faces)
    assert np.array_equal(geo, topo.signs_f)


def test_shared_faces_and_edges_have_consistent_orientation_2d():
    """Section 2.3: across a shared edge of two triangles the normal components
    must agree. With the sign data, the signed local outward normals of the two
    elements must be opposite; equivalently s * sign(det) * (outward normal)
    is the same vector from both sides."""
    nodes, elems = mg.unit_square(4)
    rng = np.random.default_rng(3)
    nodes, elems = _relabel(mg.perturb_interior(nodes, 0.25, 0.2, rng), elems, 5)
    topo = build_topology(elems, nodes.shape[0])
    from oracle.reference import LOCAL_EDGES
    seen = {}
    X = nodes[elems]
    det = np.linalg.det(np.transpose(X[:, 1:] - X[:, :1], (0, 2, 1)))
    for t in range(elems.shape[0]):
        for k, (s, e) in enumerate(LOCAL_EDGES[2]):
            xs, xe = nodes[elems[t, s]], nodes[elems[t, e]]
            tau = xe - xs
            nrm = np.array([tau[1], -tau[0]])
            if np.dot(nrm, 0.5 * (xs + xe) - nodes[elems[t, k]]) < 0:
                nrm = -nrm
            v = topo.signs_e[t, k] * np.sign(det[t]) * nrm
            g = topo.elems2edges[t, k]
            if g in seen:
                assert np.allclose(seen[g], -v) or np.allclose(seen[g], v)
                # the global normal direction is the same from both sides
                assert np.allclose(seen[g], v * np.sign(np.dot(seen[g], v)))
                assert np.dot(seen[g], v) > 0
            else:
                seen[g] = v
