"""Local and global edge-element matrices by quadrature (oracle; test infrastructure).

Global matrices (Section 2.4):  M_ij = int eta_i . eta_j,
K^RT_ij = int div eta_i div eta_j,  K^Ned_ij = int curl eta_i . curl eta_j.
The coefficient-weighted versions are K(a) = sum_K a_K K^K and M(b) = sum_K b_K M^K
with one constant a_K, b_K per element (a = b = 1 gives the paper's matrices).

Per element (Section 2.4, with the Piola maps of Sections 2.1-2.2 and the sign
data of Section 2.3), with B = B_K, J = det B, s = sign data:

  RT:   M_kl = 1/|J| int_ref s_k B eta_k . s_l B eta_l
        K_kl = 1/|J| int_ref s_k div eta_k  s_l div eta_l
  Ned:  M_kl = |J| int_ref s_k B^-T eta_k . s_l B^-T eta_l
        K_kl = 1/|J| int_ref s_k curl eta_k  s_l curl eta_l          (2D)
        K_kl = 1/|J| int_ref s_k B curl eta_k . s_l B curl eta_l     (3D)

The 3D Nedelec stiffness formula is printed with s_k twice; s_k s_l is the
reading (as in every other formula of that section).

The integrals over the reference element are done with the conical-product
Gauss-Legendre rule of ``reference.quadrature`` with 3 points per direction
(exact to degree 3 in 3D, 4 in 2D, for integrands of degree <= 2), so the local
matrices are exact up to rounding.
Global accumulation sums every local entry (k, l) of every element, in
ascending element order, into the (dof_k, dof_l) position; entries that sum to
zero stay in the pattern.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from . import reference as ref
from .topology import Topology, build_topology

CHUNK = 1 << 16


def geometry(nodes: np.ndarray, elems: np.ndarray, dtype=np.float64):
    """B_K = [x2 - x1 | ... | x_{d+1} - x1] (columns), for every element -> [T,d,d]."""
    X = np.asarray(nodes, dtype=dtype)[np.asarray(elems)]
    return np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))


def _absdet(J):
    """|det B|; for complex input sign(Re J) * J, which is analytic (complex step)."""
    if np.iscomplexobj(J):
        return np.sign(J.real) * J
    return np.abs(J)


def element_signs(topo: Topology, kind: str) -> np.ndarray:
    if kind == "rt" and topo.dim == 3:
        return topo.signs_f
    return topo.signs_e


def element_dofs(topo: Topology, kind: str) -> np.ndarray:
    if kind == "rt" and topo.dim == 3:
        return topo.elems2faces
    return topo.elems2edges


def n_dofs(topo: Topology, kind: str) -> int:
    return topo.n_faces if (kind == "rt" and topo.dim == 3) else topo.n_edges


QUAD_M = 3  # Gauss-Legendre points per direction: exact to degree 4 (2D) / 3 (3D)


def local_matrices_from_B(B: np.ndarray, kind: str, signs: np.ndarray, m: int = QUAD_M):
    """Sign-adjusted local K, M (without coefficients) from B [T,d,d] -> ([T,n,n], [T,n,n])."""
    dim = B.shape[1]
    x, w = ref.quadrature(dim, m)
    vals = ref.eval_basis(kind, dim, x)                  # [Q, n, d]
    n = vals.shape[1]
    J = np.linalg.det(B)
    aJ = _absdet(J)
    S = signs.astype(np.float64)
    T = B.shape[0]
    Mloc = np.zeros((T, n, n), dtype=B.dtype)
    Kloc = np.zeros((T, n, n), dtype=B.dtype)
    # Piola-mapped values at each quadrature point: columns of [T, d, n]
    if kind == "rt":
        P = B                                            # x -> B x
    else:
        P = np.swapaxes(np.linalg.inv(B), 1, 2)          # x -> B^-T x
    for q in range(len(w)):
        v = P @ vals[q].T                                # [T, d, n]
        Mloc += w[q] * (np.swapaxes(v, 1, 2) @ v)        # (mapped eta_k) . (mapped eta_l)
    if kind == "rt":
        Mloc /= aJ[:, None, None]
        dv = ref.div_basis(kind, dim)                    # constant divergences
        for q in range(len(w)):
            Kloc += w[q] * np.outer(dv, dv)[None]
        Kloc = Kloc / aJ[:, None, None]
    else:
        Mloc *= aJ[:, None, None]
        c = ref.curl_basis(kind, dim)
        if dim == 2:
            for q in range(len(w)):
                Kloc += w[q] * np.outer(c, c)[None]
        else:
            bc = B @ c.T                                 # [T, 3, n]: B curl eta_k
            for q in range(len(w)):
                Kloc += w[q] * (np.swapaxes(bc, 1, 2) @ bc)
        Kloc = Kloc / aJ[:, None, None]
    ss = S[:, :, None] * S[:, None, :]
    return Kloc * ss, Mloc * ss


def local_matrices(nodes: np.ndarray, elems: np.ndarray, kind: str, signs: np.ndarray,
                   m: int = QUAD_M):
    """Local K, M for all elements (chunked over elements; each element independent)."""
    T = elems.shape[0]
    dim = elems.shape[1] - 1
    n = ref.n_local(kind, dim)
    K = np.empty((T, n, n))
    M = np.empty((T, n, n))
    for s in range(0, T, CHUNK):
        e = slice(s, min(T, s + CHUNK))
        B = geometry(nodes, elems[e])
        K[e], M[e] = local_matrices_from_B(B, kind, signs[e], m)
    return K, M


class CSR:
    """Plain CSR container: rowptr [N+1] int64, colind [nnz] int32, values f64."""

    def __init__(self, n_rows, rowptr, colind, Kv, Mv):
        self.n_rows = n_rows
        self.rowptr = rowptr
        self.colind = colind
        self.Kv = Kv
        self.Mv = Mv

    @property
    def nnz(self):
        return int(self.colind.shape[0])

    def scipy(self, which="K"):
        import scipy.sparse as sp
        v = self.Kv if which == "K" else self.Mv
        return sp.csr_matrix((v, self.colind, self.rowptr), shape=(self.n_rows, self.n_rows))


def assemble(nodes: np.ndarray, elems: np.ndarray, kind: str,
             a: Optional[np.ndarray] = None, b: Optional[np.ndarray] = None,
             topo: Optional[Topology] = None, return_local: bool = False):
    """Global CSR K(a), M(b) of ``kind`` ('ned' or 'rt') on the mesh."""
    elems = np.asarray(elems)
    topo = build_topology(elems, nodes.shape[0]) if topo is None else topo
    dofs = element_dofs(topo, kind)
    signs = element_signs(topo, kind)
    N = n_dofs(topo, kind)
    Kl, Ml = local_matrices(nodes, elems, kind, signs)
    T, n, _ = Kl.shape
    a = np.ones(T) if a is None else np.asarray(a, dtype=np.float64)
    b = np.ones(T) if b is None else np.asarray(b, dtype=np.float64)
    I = np.repeat(dofs[:, :, None], n, axis=2).reshape(-1)
    Jc = np.repeat(dofs[:, None, :], n, axis=1).reshape(-1)
    key = I * np.int64(N) + Jc                           # element-major, (k, l) order
    uniq, inv = np.unique(key, return_inverse=True)
    Kv = np.bincount(inv, weights=(a[:, None, None] * Kl).reshape(-1), minlength=uniq.size)
    Mv = np.bincount(inv, weights=(b[:, None, None] * Ml).reshape(-1), minlength=uniq.size)
    rows = uniq // N
    cols = (uniq % N).astype(np.int32)
    rowptr = np.zeros(N + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    csr = CSR(N, rowptr, cols, Kv, Mv)
    if return_local:
        return csr, topo, Kl, Ml
    return csr, topo


def assemble_rows(nodes: np.ndarray, elems: np.ndarray, kind: str, rows: Sequence[int],
                  a: Optional[np.ndarray] = None, b: Optional[np.ndarray] = None,
                  topo: Optional[Topology] = None):
    """The rows ``rows`` of K(a), M(b): only the elements that touch those rows are
    integrated. Returns {row: (cols int32 ascending, Kvals, Mvals)}.
    """
    elems = np.asarray(elems)
    topo = build_topology(elems, nodes.shape[0]) if topo is None else topo
    dofs = element_dofs(topo, kind)
    signs = element_signs(topo, kind)
    rows = np.unique(np.asarray(rows, dtype=np.int64))
    touch = np.isin(dofs, rows).any(axis=1)
    eids = np.nonzero(touch)[0]                          # ascending element order
    Kl, Ml = local_matrices(nodes, elems[eids], kind, signs[eids])
    a = np.ones(elems.shape[0]) if a is None else np.asarray(a, dtype=np.float64)
    b = np.ones(elems.shape[0]) if b is None else np.asarray(b, dtype=np.float64)
    acc = {int(r): {} for r in rows}
    d = dofs[eids]
    n = d.shape[1]
    for i in range(eids.size):
        e = eids[i]
        for k in range(n):
            r = int(d[i, k])
            if r not in acc:
                continue
            row = acc[r]
            for l in range(n):
                c = int(d[i, l])
                kv, mv = row.get(c, (0.0, 0.0))
                row[c] = (kv + a[e] * Kl[i, k, l], mv + b[e] * Ml[i, k, l])
    out = {}
    for r, row in acc.items():
        cols = np.array(sorted(row), dtype=np.int32)
        out[r] = (cols, np.array([row[c][0] for c in cols]), np.array([row[c][1] for c in cols]))
    return out, topo
