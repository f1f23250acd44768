"""Reference elements, reference bases and quadrature (oracle; test infrastructure).

Reference configurations (Section 2, Figure 1): the unit triangle with nodes
1=(0,0), 2=(1,0), 3=(0,1) and the unit tetrahedron with nodes 1=0, 2=e1, 3=e2,
4=e3. Local numbers here are 0-based (node ``i`` of the paper is ``i-1``).

Every reference basis function of the lowest-order elements is affine, so it is
stored as ``eta_k(x) = P_k x + q_k``. The tables below are the printed reference
bases of Section 2.1 (Raviart-Thomas) and Section 2.2 (Nedelec) written in that
form. div and curl of an affine field are read off ``P``: ``div = trace(P)``,
3D ``curl = (P32 - P23, P13 - P31, P21 - P12)`` and 2D scalar
``curl = P21 - P12`` (definitions at the start of Section 2).
"""
from __future__ import annotations

import numpy as np

# --- reference vertices (Figure 1) -------------------------------------------------
REF_NODES = {
    2: np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]),
    3: np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]),
}
REF_VOLUME = {2: 0.5, 3: 1.0 / 6.0}

# --- local edges / faces (Figure 1) -----------------------------------------------
# Directed local edges (start, end), 0-based.
#  2D: edge k is opposite node k and runs from node k+1 to node k+2 (cyclically),
#      which is the rule stated for the sign data in Section 3.
#  3D: the arrows of Figure 1: 1->2, 1->3, 1->4, 2->3, 3->4, 4->2.
LOCAL_EDGES = {
    2: ((1, 2), (2, 0), (0, 1)),
    3: ((0, 1), (0, 2), (0, 3), (1, 2), (2, 3), (3, 1)),
}
# 3D faces: face k is opposite node 4-k (0-based: face k opposite node 3-k),
# normals pointing outwards (Figure 1).
LOCAL_FACES = ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3))
FACE_OPPOSITE = (3, 2, 1, 0)


def _affine(P, q):
    return np.array(P, dtype=np.float64), np.array(q, dtype=np.float64)


# --- Raviart-Thomas reference basis (Section 2.1) ---------------------------------
# 2D: eta1 = (x1, x2), eta2 = (x1 - 1, x2), eta3 = (x1, x2 - 1)
RT_BASIS_2D = [
    _affine([[1, 0], [0, 1]], [0, 0]),
    _affine([[1, 0], [0, 1]], [-1, 0]),
    _affine([[1, 0], [0, 1]], [0, -1]),
]
# 3D: eta1 = (x1, x2, x3 - 1), eta2 = (x1, x2 - 1, x3), eta3 = (x1 - 1, x2, x3),
#     eta4 = (x1, x2, x3)
_I3 = [[1, 0, 0], [0, 1, 0], [0, 0, 1]]
RT_BASIS_3D = [
    _affine(_I3, [0, 0, -1]),
    _affine(_I3, [0, -1, 0]),
    _affine(_I3, [-1, 0, 0]),
    _affine(_I3, [0, 0, 0]),
]

# --- Nedelec reference basis (Section 2.2) ----------------------------------------
# 2D: eta1 = (-x2, x1), eta2 = (-x2, x1 - 1), eta3 = (1 - x2, x1)
NED_BASIS_2D = [
    _affine([[0, -1], [1, 0]], [0, 0]),
    _affine([[0, -1], [1, 0]], [0, -1]),
    _affine([[0, -1], [1, 0]], [1, 0]),
]
# 3D: eta1 = (1 - x3 - x2, x1, x1), eta2 = (x2, 1 - x3 - x1, x2),
#     eta3 = (x3, x3, 1 - x2 - x1), eta4 = (-x2, x1, 0), eta5 = (0, -x3, x2),
#     eta6 = (x3, 0, -x1)
NED_BASIS_3D = [
    _affine([[0, -1, -1], [1, 0, 0], [1, 0, 0]], [1, 0, 0]),
    _affine([[0, 1, 0], [-1, 0, -1], [0, 1, 0]], [0, 1, 0]),
    _affine([[0, 0, 1], [0, 0, 1], [-1, -1, 0]], [0, 0, 1]),
    _affine([[0, -1, 0], [1, 0, 0], [0, 0, 0]], [0, 0, 0]),
    _affine([[0, 0, 0], [0, 0, -1], [0, 1, 0]], [0, 0, 0]),
    _affine([[0, 0, 1], [0, 0, 0], [-1, 0, 0]], [0, 0, 0]),
]


def basis(kind: str, dim: int):
    """List of (P, q) for the reference basis of ``kind`` ('rt' or 'ned') in ``dim``."""
    if kind == "rt":
        return RT_BASIS_2D if dim == 2 else RT_BASIS_3D
    if kind == "ned":
        return NED_BASIS_2D if dim == 2 else NED_BASIS_3D
    raise ValueError(kind)


def n_local(kind: str, dim: int) -> int:
    return len(basis(kind, dim))


def eval_basis(kind: str, dim: int, x: np.ndarray) -> np.ndarray:
    """Values of all reference basis functions at points ``x`` [Q,d] -> [Q, nb, d]."""
    out = []
    for P, q in basis(kind, dim):
        out.append(x @ P.T + q)
    return np.stack(out, axis=1)


def div_basis(kind: str, dim: int) -> np.ndarray:
    """Constant divergence of each reference basis function -> [nb]."""
    return np.array([np.trace(P) for P, _ in basis(kind, dim)])


def curl_basis(kind: str, dim: int) -> np.ndarray:
    """Constant curl of each reference basis function: [nb] (2D scalar) or [nb,3]."""
    out = []
    for P, _ in basis(kind, dim):
        if dim == 2:
            out.append(P[1, 0] - P[0, 1])
        else:
            out.append([P[2, 1] - P[1, 2], P[0, 2] - P[2, 0], P[1, 0] - P[0, 1]])
    return np.array(out, dtype=np.float64)


# --- quadrature -------------------------------------------------------------------
def gauss_legendre_01(m: int):
    """m-point Gauss-Legendre rule on [0,1]."""
    x, w = np.polynomial.legendre.leggauss(m)
    return 0.5 * (x + 1.0), 0.5 * w


def quadrature(dim: int, m: int = 4):
    """Conical-product (collapsed coordinate) Gauss-Legendre rule on the reference
    simplex: m^dim points, exact for polynomials of total degree <= 2m - dim.

    2D: x1 = u, x2 = v (1 - u), dx = (1 - u) du dv.
    3D: x1 = u, x2 = v (1 - u), x3 = w (1 - u)(1 - v), dx = (1-u)^2 (1-v) du dv dw.
    Returns (points [Q,d], weights [Q]).
    """
    t, w = gauss_legendre_01(m)
    if dim == 2:
        U, V = np.meshgrid(t, t, indexing="ij")
        WU, WV = np.meshgrid(w, w, indexing="ij")
        x1 = U
        x2 = V * (1.0 - U)
        W = WU * WV * (1.0 - U)
        return np.stack([x1.ravel(), x2.ravel()], axis=1), W.ravel()
    if dim == 3:
        U, V, Z = np.meshgrid(t, t, t, indexing="ij")
        WU, WV, WZ = np.meshgrid(w, w, w, indexing="ij")
        x1 = U
        x2 = V * (1.0 - U)
        x3 = Z * (1.0 - U) * (1.0 - V)
        W = WU * WV * WZ * (1.0 - U) ** 2 * (1.0 - V)
        return np.stack([x1.ravel(), x2.ravel(), x3.ravel()], axis=1), W.ravel()
    raise ValueError(dim)
