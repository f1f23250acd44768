"""Gradient of L = sum_p gK[p] K(a)[p] + sum_p gM[p] M(b)[p] (oracle; test infrastructure).

For L = u^T (K(a) + M(b)) u the weights are gK[p] = gM[p] = u_row(p) u_col(p).

* dL/da_K = sum_kl gK[pos(K,k,l)] K~^K_kl   and   dL/db_K likewise with M~,
  where K~, M~ are the local matrices without coefficient (exact: linear in a, b).
* dL/dx for every vertex coordinate: the local matrices of each element are
  differentiated by the complex-step method (Squire & Trapp, SIAM Rev. 1998):
  f'(x) = Im f(x + i h) / h with h = 1e-30, which has no subtractive
  cancellation. |det B| is replaced by sign(Re det B) det B so the quadrature
  formulas stay analytic. Per-element vertex derivatives are summed into the
  vertices in ascending element order.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from .assembly import (CSR, element_dofs, element_signs, geometry, local_matrices,
                       local_matrices_from_B)
from .topology import Topology

H_CS = 1e-30
CHUNK = 1 << 16


def positions(csr: CSR, dofs: np.ndarray) -> np.ndarray:
    """CSR position of every local entry (k, l) of every element -> [T, n, n] int64,
    by binary search of the keys I*N + J in the row-major sorted pattern."""
    n_rows = csr.n_rows
    T, n = dofs.shape
    rows = np.repeat(np.arange(n_rows, dtype=np.int64), np.diff(csr.rowptr))
    keys = rows * np.int64(n_rows) + csr.colind.astype(np.int64)
    I = np.repeat(dofs[:, :, None], n, axis=2).astype(np.int64)
    Jc = np.repeat(dofs[:, None, :], n, axis=1).astype(np.int64)
    q = I * np.int64(n_rows) + Jc
    pos = np.searchsorted(keys, q.reshape(-1))
    assert np.array_equal(keys[pos], q.reshape(-1))
    return pos.reshape(T, n, n)


def grad_coefficients(nodes, elems, kind, topo: Topology, pos: np.ndarray,
                      gK: np.ndarray, gM: np.ndarray):
    """dL/da, dL/db per element (exact)."""
    Kl, Ml = local_matrices(nodes, elems, kind, element_signs(topo, kind))
    ga = np.einsum("tkl,tkl->t", gK[pos], Kl)
    gb = np.einsum("tkl,tkl->t", gM[pos], Ml)
    return ga, gb


def grad_nodes(nodes, elems, kind, topo: Topology, pos: np.ndarray, gK: np.ndarray,
               gM: np.ndarray, a: Optional[np.ndarray] = None, b: Optional[np.ndarray] = None):
    """dL/dx for every vertex coordinate by complex-step differentiation -> [V, d]."""
    elems = np.asarray(elems)
    T = elems.shape[0]
    dim = elems.shape[1] - 1
    a = np.ones(T) if a is None else np.asarray(a, dtype=np.float64)
    b = np.ones(T) if b is None else np.asarray(b, dtype=np.float64)
    signs = element_signs(topo, kind)
    per_elem = np.zeros((T, dim + 1, dim))
    for s in range(0, T, CHUNK):
        e = slice(s, min(T, s + CHUNK))
        X = np.asarray(nodes, dtype=np.complex128)[elems[e]]          # [t, d+1, d]
        GK = gK[pos[e]]
        GM = gM[pos[e]]
        for v in range(dim + 1):
            for c in range(dim):
                Xp = X.copy()
                Xp[:, v, c] += 1j * H_CS
                B = np.transpose(Xp[:, 1:, :] - Xp[:, :1, :], (0, 2, 1))
                Kc, Mc = local_matrices_from_B(B, kind, signs[e])
                dK = Kc.imag / H_CS
                dM = Mc.imag / H_CS
                per_elem[e, v, c] = (a[e] * np.einsum("tkl,tkl->t", GK, dK)
                                     + b[e] * np.einsum("tkl,tkl->t", GM, dM))
    g = np.zeros((nodes.shape[0], dim))
    for v in range(dim + 1):
        np.add.at(g, elems[:, v], per_elem[:, v, :])
    return g


def loss(csr: CSR, u: np.ndarray) -> float:
    """L = u^T K u + u^T M u for the CSR matrices."""
    rows = np.repeat(np.arange(csr.n_rows), np.diff(csr.rowptr))
    w = u[rows] * u[csr.colind]
    return float(np.dot(w, csr.Kv) + np.dot(w, csr.Mv))


def quadratic_weights(csr: CSR, u: np.ndarray) -> np.ndarray:
    """gK[p] = gM[p] = u_row(p) u_col(p): the weights of L = u^T (K + M) u."""
    rows = np.repeat(np.arange(csr.n_rows), np.diff(csr.rowptr))
    return u[rows] * u[csr.colind]
