"""Minimisation of the functional majorant (Section 4.1) (oracle; test infrastructure).

Poisson problem -Lap u = f in the unit square / cube, u = 0 on the boundary,
with the bubble solution u(x) = prod_i x_i (x_i - 1) of the example, so
f = -Lap u = -2 sum_i prod_{j != i} x_j (x_j - 1).

* v: the approximation from linear nodal (P1) elements: stiffness
  K_ij = int grad(lambda_i) . grad(lambda_j), load F_i = int f lambda_i (by the
  quadrature of ``integrate``), boundary nodes fixed to 0, direct solve.
* For fixed beta the majorant is a quadratic functional of y in H(div); its
  minimiser over the Raviart-Thomas space (the discretised problem of
  Section 4.1) solves
      ((1 + beta) C^2 K_RT + (1 + 1/beta) M_RT) y
          = -(1 + beta) C^2 int f div phi_i + (1 + 1/beta) int grad v . phi_i,
  with K_RT, M_RT from ``assembly.assemble`` and the global Raviart-Thomas
  basis phi_k = s_k B_K eta^_k / det B_K on each element (the contravariant
  Piola map of Section 2.1 with the signed determinant, the one the sign data
  of Section 2.3 belong to: with it the normal component of a discrete field
  is continuous across interior facets).
* beta is then updated to ||grad v - y|| / (C ||div y + f||) (Algorithm 1 of
  Section 4.1), starting from beta = 1, until the majorant changes by less than
  1e-4 relative to its previous value.
* The reported values are, per iteration, beta, the majorant
  M = sqrt((1 + 1/beta) ||grad v - y||^2 + (1 + beta) C^2 ||div y + f||^2)
  (the paper's tables print this square root: it decreases like h, as the
  error does) and the efficiency index M / ||grad(u - v)||.
* C is the Friedrichs constant of the domain, 1 / (pi sqrt(d)) for the unit
  square (d = 2) and cube (d = 3) (the paper does not print it; this is its
  sharp value, 1 / sqrt of the first Dirichlet eigenvalue d pi^2).
"""
from __future__ import annotations

import numpy as np

from . import reference as ref
from .assembly import assemble, element_dofs, element_signs
from .integrate import DEFAULT_M, affine_transformations


def bubble_u(X):
    return np.prod(X * (X - 1.0), axis=1)


def bubble_grad_u(X):
    d = X.shape[1]
    g = np.empty_like(X)
    for i in range(d):
        others = np.prod(np.delete(X * (X - 1.0), i, axis=1), axis=1)
        g[:, i] = (2.0 * X[:, i] - 1.0) * others
    return g


def bubble_f(X):
    """f = -Lap u for the bubble u."""
    d = X.shape[1]
    s = np.zeros(X.shape[0])
    for i in range(d):
        s -= 2.0 * np.prod(np.delete(X * (X - 1.0), i, axis=1), axis=1)
    return s


def friedrichs_constant(dim: int) -> float:
    return 1.0 / (np.pi * np.sqrt(dim))


def boundary_nodes(nodes: np.ndarray, elems: np.ndarray) -> np.ndarray:
    """Nodes of the boundary facets (facets that belong to one element)."""
    dim = elems.shape[1] - 1
    e = np.asarray(elems, dtype=np.int64)
    facets = np.sort(np.concatenate([np.delete(e, k, axis=1) for k in range(dim + 1)]), axis=1)
    uniq, cnt = np.unique(facets, axis=0, return_counts=True)
    flag = np.zeros(nodes.shape[0], dtype=bool)
    flag[uniq[cnt == 1].reshape(-1)] = True
    return flag


def p1_gradients(nodes, elems):
    """grad lambda_a of every element -> [T, d+1, d] (rows of B_K^-1 for a >= 1,
    minus their sum for a = 0), and det B_K."""
    B, _, det = affine_transformations(nodes, elems)
    Binv = np.linalg.inv(B)
    G = np.concatenate([-Binv.sum(axis=1, keepdims=True), Binv], axis=1)
    return G, det


def p1_system(nodes, elems, f=bubble_f, m=None):
    """P1 stiffness (scipy CSR, no boundary condition) and load vector
    int f lambda_i (element sums added in ascending element order)."""
    import scipy.sparse as sp
    dim = elems.shape[1] - 1
    m = DEFAULT_M[dim] if m is None else m
    G, det = p1_gradients(nodes, elems)
    vol = np.abs(det) * ref.REF_VOLUME[dim]
    Kl = vol[:, None, None] * np.einsum("tad,tbd->tab", G, G)
    B, b, _ = affine_transformations(nodes, elems)
    xq, wq = ref.quadrature(dim, m)
    Fl = np.zeros((elems.shape[0], dim + 1))
    for i in range(len(wq)):
        X = np.einsum("tij,j->ti", B, xq[i]) + b
        lam = np.concatenate([[1.0 - xq[i].sum()], xq[i]])
        Fl += wq[i] * np.abs(det)[:, None] * f(X)[:, None] * lam[None, :]
    V = nodes.shape[0]
    e = np.asarray(elems, dtype=np.int64)
    I = np.repeat(e, dim + 1, axis=1).reshape(-1)
    J = np.tile(e, (1, dim + 1)).reshape(-1)
    K = sp.csr_matrix((Kl.reshape(-1), (I, J)), shape=(V, V))
    K.sum_duplicates()
    F = np.bincount(e.reshape(-1), weights=Fl.reshape(-1), minlength=V)
    return K, F


def p1_solve(nodes, elems, f=bubble_f, m=None):
    """v: P1 solution with v = 0 at the boundary nodes (direct solve)."""
    import scipy.sparse.linalg as spla
    K, F = p1_system(nodes, elems, f, m)
    free = ~boundary_nodes(nodes, elems)
    v = np.zeros(nodes.shape[0])
    v[free] = spla.spsolve(K[free][:, free].tocsc(), F[free])
    return v


def grad_error(nodes, elems, v, grad_u=bubble_grad_u, m=None):
    """||grad(u - v)|| for the P1 field v."""
    dim = elems.shape[1] - 1
    m = DEFAULT_M[dim] if m is None else m
    G, det = p1_gradients(nodes, elems)
    gv = np.einsum("ta,tad->td", v[elems], G)
    B, b, _ = affine_transformations(nodes, elems)
    xq, wq = ref.quadrature(dim, m)
    s = 0.0
    for i in range(len(wq)):
        X = np.einsum("tij,j->ti", B, xq[i]) + b
        s += np.sum(wq[i] * np.abs(det) * np.sum((grad_u(X) - gv) ** 2, axis=1))
    return float(np.sqrt(s))


def rt_basis_at(B, det, xq, dim):
    """s-free Raviart-Thomas basis B eta^_k(x^) / det B at one reference point
    -> [T, n, d]; the divergence of each is div^eta^_k / det B."""
    vals = ref.eval_basis("rt", dim, xq[None, :])[0]
    return np.einsum("tij,kj->tki", B, vals) / det[:, None, None]


def rt_loads(nodes, elems, topo, v, f=bubble_f, m=None):
    """(int f div phi_i, int grad v . phi_i) over the global RT basis."""
    dim = elems.shape[1] - 1
    m = DEFAULT_M[dim] if m is None else m
    B, b, det = affine_transformations(nodes, elems)
    G, _ = p1_gradients(nodes, elems)
    gv = np.einsum("ta,tad->td", v[elems], G)
    S = element_signs(topo, "rt").astype(np.float64)
    D = element_dofs(topo, "rt")
    divref = ref.div_basis("rt", dim)
    xq, wq = ref.quadrature(dim, m)
    ld = np.zeros(D.shape)
    lg = np.zeros(D.shape)
    for i in range(len(wq)):
        X = np.einsum("tij,j->ti", B, xq[i]) + b
        w = wq[i] * np.abs(det)
        ld += w[:, None] * f(X)[:, None] * (divref[None, :] / det[:, None])
        lg += w[:, None] * np.einsum("tki,ti->tk", rt_basis_at(B, det, xq[i], dim), gv)
    n = topo.n_faces if dim == 3 else topo.n_edges
    Fd = np.bincount(D.reshape(-1), weights=(ld * S).reshape(-1), minlength=n)
    Fg = np.bincount(D.reshape(-1), weights=(lg * S).reshape(-1), minlength=n)
    return Fd, Fg


def majorant_terms(nodes, elems, topo, v, y, f=bubble_f, m=None):
    """(||grad v - y||^2, ||div y + f||^2) for the P1 field v and the RT field y."""
    dim = elems.shape[1] - 1
    m = DEFAULT_M[dim] if m is None else m
    B, b, det = affine_transformations(nodes, elems)
    G, _ = p1_gradients(nodes, elems)
    gv = np.einsum("ta,tad->td", v[elems], G)
    S = element_signs(topo, "rt").astype(np.float64)
    ye = np.asarray(y)[element_dofs(topo, "rt")] * S
    divy = (ye @ ref.div_basis("rt", dim)) / det
    xq, wq = ref.quadrature(dim, m)
    a2 = 0.0
    b2 = 0.0
    for i in range(len(wq)):
        X = np.einsum("tij,j->ti", B, xq[i]) + b
        yh = np.einsum("tki,tk->ti", rt_basis_at(B, det, xq[i], dim), ye)
        w = wq[i] * np.abs(det)
        a2 += np.sum(w * np.sum((gv - yh) ** 2, axis=1))
        b2 += np.sum(w * (divy + f(X)) ** 2)
    return float(a2), float(b2)


def minimise(nodes, elems, beta0=1.0, tol=1e-4, max_iter=20, m=None):
    """Algorithm 1 of Section 4.1 on one mesh. Returns a dict: the P1 solution
    v, its error ||grad(u - v)||, and per iteration (beta, majorant M,
    efficiency index, y)."""
    import scipy.sparse.linalg as spla
    dim = elems.shape[1] - 1
    C = friedrichs_constant(dim)
    v = p1_solve(nodes, elems, m=m)
    err = grad_error(nodes, elems, v, m=m)
    csr, topo = assemble(nodes, elems, "rt")
    K, M = csr.scipy("K"), csr.scipy("M")
    Fd, Fg = rt_loads(nodes, elems, topo, v, m=m)
    beta = beta0
    iters = []
    prev = None
    for _ in range(max_iter):
        cK = (1.0 + beta) * C * C
        cM = 1.0 + 1.0 / beta
        y = spla.spsolve((cK * K + cM * M).tocsc(), -cK * Fd + cM * Fg)
        a2, b2 = majorant_terms(nodes, elems, topo, v, y, m=m)
        Mval = float(np.sqrt(cM * a2 + cK * b2))
        iters.append(dict(beta=beta, majorant=Mval, ieff=Mval / err, y=y, terms=(a2, b2)))
        if prev is not None and abs(prev - Mval) / prev < tol:
            break
        prev = Mval
        beta = float(np.sqrt(a2) / (C * np.sqrt(b2)))
    return dict(v=v, error=err, topo=topo, csr=csr, iterations=iters, Fd=Fd, Fg=Fg)
