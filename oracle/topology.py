"""Global numbering of edges/faces and orientation sign data (oracle; test infrastructure).

Section 3 defines the mesh structures: ``edges2nodes`` / ``faces2nodes`` list the
global edges / faces by their nodes, the row index is the global degree of
freedom, and ``elems2edges`` / ``elems2faces`` give each element's global dofs
in local order. The paper does not fix the order of the rows; the reading used
here (and by the GPU library) is: each edge is the sorted node pair (lo, hi),
each face the sorted triple (a, b, c), and rows are in lexicographic order of
these tuples.

Sign data (Section 2.3 and Section 3):

* Edges (Nedelec in 2D and 3D, Raviart-Thomas in 2D): local edge k directed
  from its start to its end node (Figure 1) gets +1 if the global index of the
  start node is larger than that of the end node and -1 otherwise. Section 3
  states this rule for 2D; the same rule with the 3D arrows of Figure 1 is the
  3D reading.
* Faces (Raviart-Thomas in 3D, not stated in the paper): with (a, b, c) the
  sorted global nodes of local face k and p the opposite node, the sign is
  minus the parity of the permutation that takes the element's local node order
  to the order (a, b, c, p). ``signs_faces_geometric`` is the det-based
  definition of Section 2.3 (sign of det B_K times the sign of the outward
  normal against the global face normal (x_b - x_a) x (x_c - x_a)); tests check
  the two agree.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from .reference import LOCAL_EDGES, LOCAL_FACES, FACE_OPPOSITE


@dataclass
class Topology:
    dim: int
    n_nodes: int
    edges2nodes: np.ndarray            # [E,2] int64, lo < hi, lexicographic rows
    elems2edges: np.ndarray            # [T,3|6] int64
    signs_e: np.ndarray                # [T,3|6] int8
    faces2nodes: Optional[np.ndarray]  # [F,3] int64 (3D)
    elems2faces: Optional[np.ndarray]  # [T,4] int64 (3D)
    signs_f: Optional[np.ndarray]      # [T,4] int8 (3D)

    @property
    def n_edges(self) -> int:
        return self.edges2nodes.shape[0]

    @property
    def n_faces(self) -> int:
        return 0 if self.faces2nodes is None else self.faces2nodes.shape[0]


def _unique_rows_lex(cols):
    """Unique rows of the integer columns ``cols`` (each [n], values < 2^31) in
    lexicographic order, and for every input row the index of its unique row.
    A lexicographic sort followed by "keep the first of each run"."""
    order = np.lexsort(tuple(reversed(cols)))           # primary key = cols[0]
    srt = [c[order] for c in cols]
    head = np.ones(order.size, dtype=bool)
    if order.size > 1:
        diff = np.zeros(order.size - 1, dtype=bool)
        for c in srt:
            diff |= c[1:] != c[:-1]
        head[1:] = diff
    rank = np.cumsum(head) - 1
    inv = np.empty(order.size, dtype=np.int64)
    inv[order] = rank
    uniq = np.stack([c[head] for c in srt], axis=1)
    return uniq, inv


def get_edges(elems: np.ndarray):
    """Unique edges (lexicographic rows of sorted node pairs) and the element->edge map."""
    dim = elems.shape[1] - 1
    e = np.asarray(elems, dtype=np.int64)
    ne = len(LOCAL_EDGES[dim])
    s = np.stack([e[:, a] for a, _ in LOCAL_EDGES[dim]], axis=1).reshape(-1)
    t = np.stack([e[:, b] for _, b in LOCAL_EDGES[dim]], axis=1).reshape(-1)
    lo, hi = np.minimum(s, t), np.maximum(s, t)           # (lo, hi) per local edge
    uniq, inv = _unique_rows_lex([lo, hi])
    return uniq, inv.reshape(e.shape[0], ne)


def get_faces(elems: np.ndarray):
    """Unique faces (lexicographic rows of sorted node triples) and the element->face map."""
    e = np.asarray(elems, dtype=np.int64)
    tri = np.sort(np.stack([e[:, list(f)] for f in LOCAL_FACES], axis=1), axis=2).reshape(-1, 3)
    uniq, inv = _unique_rows_lex([tri[:, 0], tri[:, 1], tri[:, 2]])
    return uniq, inv.reshape(e.shape[0], 4)


def signs_edges(elems: np.ndarray) -> np.ndarray:
    """+1 where the global start node of a local edge is larger than its end node."""
    dim = elems.shape[1] - 1
    e = np.asarray(elems, dtype=np.int64)
    cols = []
    for s, t in LOCAL_EDGES[dim]:
        cols.append(np.where(e[:, s] > e[:, t], 1, -1))
    return np.stack(cols, axis=1).astype(np.int8)


def _perm_parity(p: np.ndarray) -> np.ndarray:
    """Parity (+1 even, -1 odd) of each row of ``p`` (a permutation of 0..n-1), by
    counting inversions."""
    n = p.shape[1]
    inv = np.zeros(p.shape[0], dtype=np.int64)
    for i in range(n):
        for j in range(i + 1, n):
            inv += (p[:, i] > p[:, j])
    return np.where(inv % 2 == 0, 1, -1)


def signs_faces(elems: np.ndarray) -> np.ndarray:
    """Minus the parity of local order -> (sorted face nodes, opposite node)."""
    e = np.asarray(elems, dtype=np.int64)
    T = e.shape[0]
    out = np.empty((T, 4), dtype=np.int8)
    for k, f in enumerate(LOCAL_FACES):
        loc = np.array(f)
        g = e[:, loc]                                    # global ids of the face nodes
        order = np.argsort(g, axis=1, kind="stable")     # local positions in sorted order
        sorted_loc = loc[order]                          # local node numbers of (a, b, c)
        perm = np.concatenate([sorted_loc, np.full((T, 1), FACE_OPPOSITE[k])], axis=1)
        out[:, k] = -_perm_parity(perm)
    return out


def signs_faces_geometric(nodes: np.ndarray, elems: np.ndarray, faces2nodes, elems2faces) -> np.ndarray:
    """Det-based face signs: sign(det B_K) * sign(n_out . n_f), n_f = (x_b-x_a) x (x_c-x_a)."""
    X = nodes[elems]
    B = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))
    detB = np.linalg.det(B)
    out = np.empty((elems.shape[0], 4), dtype=np.int8)
    centroid = X.mean(axis=1)
    for k, f in enumerate(LOCAL_FACES):
        fn = faces2nodes[elems2faces[:, k]]
        xa, xb, xc = nodes[fn[:, 0]], nodes[fn[:, 1]], nodes[fn[:, 2]]
        nf = np.cross(xb - xa, xc - xa)
        # outward direction: from the element centroid towards the face
        outward = np.einsum("ti,ti->t", nf, xa - centroid)
        out[:, k] = (np.sign(detB) * np.sign(outward)).astype(np.int8)
    return out


def build_topology(elems: np.ndarray, n_nodes: Optional[int] = None) -> Topology:
    dim = elems.shape[1] - 1
    n_nodes = int(elems.max()) + 1 if n_nodes is None else n_nodes
    e2n, el2e = get_edges(elems)
    se = signs_edges(elems)
    f2n = el2f = sf = None
    if dim == 3:
        f2n, el2f = get_faces(elems)
        sf = signs_faces(elems)
    return Topology(dim, n_nodes, e2n, el2e, se, f2n, el2f, sf)


def brute_force_topology(elems):
    """Pure-Python set/dict version of ``build_topology`` for tiny meshes."""
    dim = len(elems[0]) - 1
    edge_set = set()
    face_set = set()
    for el in elems:
        for s, t in LOCAL_EDGES[dim]:
            edge_set.add(tuple(sorted((int(el[s]), int(el[t])))))
        if dim == 3:
            for f in LOCAL_FACES:
                face_set.add(tuple(sorted(int(el[i]) for i in f)))
    edges = sorted(edge_set)
    eid = {e: i for i, e in enumerate(edges)}
    faces = sorted(face_set)
    fid = {f: i for i, f in enumerate(faces)}
    el2e = [[eid[tuple(sorted((int(el[s]), int(el[t]))))] for s, t in LOCAL_EDGES[dim]] for el in elems]
    el2f = [[fid[tuple(sorted(int(el[i]) for i in f))] for f in LOCAL_FACES] for el in elems] if dim == 3 else None
    return edges, el2e, faces, el2f
