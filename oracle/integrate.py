"""Vectorised integration of a function over a mesh (oracle; test infrastructure).

Section 3.1 of the paper computes the squared L2 norm of a function f in two
steps: the affine maps F_K(x^) = B_K x^ + b_K of all elements (B_K, b_K and
det B_K), then a loop over the points of a quadrature rule on the reference
element (not over the elements): at point i every element's image F_K(x^_i) is
formed at once and w_i |det B_K| f(F_K(x^_i))^2 is added to that element's
sum. The element sums are ||f||_K^2; their total is ||f||^2.

The quadrature rule is the conical-product Gauss-Legendre rule of
``reference.quadrature``. The paper uses rules of order 6 (exact for
polynomials of degree 6, so ||f||^2 is exact for cubic f); the default here is
the smallest m whose rule reaches degree 6: m = 4 in 2D (degree 6), m = 5 in 3D
(degree 7).
"""
from __future__ import annotations

from typing import Callable

import numpy as np

from . import reference as ref
from .assembly import element_dofs, element_signs

DEFAULT_M = {2: 4, 3: 5}


def affine_transformations(nodes: np.ndarray, elems: np.ndarray):
    """B_K [T,d,d] (columns x_{i+1} - x_1), b_K [T,d] (= x_1) and det B_K [T]
    (Section 3.1, `affine_transformations`)."""
    X = np.asarray(nodes, dtype=np.float64)[np.asarray(elems)]
    B = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))
    b = X[:, 0, :].copy()
    return B, b, np.linalg.det(B)


def integrate_elements(nodes: np.ndarray, elems: np.ndarray, g: Callable, m: int | None = None):
    """Per-element integrals int_K g(x) dx -> [T]. ``g`` maps points [T,d] to
    values [T] (it is called once per quadrature point with every element's
    image of that point)."""
    dim = elems.shape[1] - 1
    m = DEFAULT_M[dim] if m is None else m
    B, b, det = affine_transformations(nodes, elems)
    absdet = np.abs(det)
    xq, wq = ref.quadrature(dim, m)
    acc = np.zeros(elems.shape[0])
    for i in range(len(wq)):
        X = np.einsum("tij,j->ti", B, xq[i]) + b   # F_K(x^_i) for every K
        acc += wq[i] * absdet * g(X)
    return acc


def norm_L2_squared(nodes: np.ndarray, elems: np.ndarray, f: Callable, m: int | None = None):
    """(per-element ||f||_K^2 [T], total ||f||^2) of a scalar or vector
    function ``f`` (points [T,d] -> [T] or [T,c]; for a vector function the
    squared Euclidean norm is integrated)."""
    def sq(X):
        v = np.asarray(f(X), dtype=np.float64)
        return v * v if v.ndim == 1 else np.sum(v * v, axis=1)
    per = integrate_elements(nodes, elems, sq, m)
    return per, float(np.sum(per))


def _ned_basis_at(B_inv_T: np.ndarray, xq: np.ndarray, dim: int) -> np.ndarray:
    """Covariant Piola images B_K^-T eta^_k(x^) of the reference Nedelec basis
    (Section 2.2) at one reference point, for every element -> [T, n, d]."""
    vals = ref.eval_basis("ned", dim, xq[None, :])[0]            # [n, d]
    return np.einsum("tij,kj->tki", B_inv_T, vals)


def load_vector_ned(nodes, elems, topo, F: Callable, m: int | None = None):
    """f_i = int F . eta_i over the global Nedelec basis (Sections 2.2-2.3):
    per element, sum over the quadrature points of
    w_q |det B_K| F(F_K(x^_q)) . s_k B_K^-T eta^_k(x^_q); then the local values
    are added to their edges in ascending element order."""
    dim = elems.shape[1] - 1
    m = DEFAULT_M[dim] if m is None else m
    B, b, det = affine_transformations(nodes, elems)
    BmT = np.swapaxes(np.linalg.inv(B), 1, 2)
    S = element_signs(topo, "ned").astype(np.float64)
    D = element_dofs(topo, "ned")
    xq, wq = ref.quadrature(dim, m)
    loc = np.zeros(D.shape)
    for i in range(len(wq)):
        X = np.einsum("tij,j->ti", B, xq[i]) + b
        phi = _ned_basis_at(BmT, xq[i], dim)
        loc += wq[i] * np.abs(det)[:, None] * np.einsum("tki,ti->tk", phi, F(X))
    loc *= S
    return np.bincount(D.reshape(-1), weights=loc.reshape(-1), minlength=topo.n_edges)


def hcurl_error_ned(nodes, elems, topo, v, E: Callable, curlE: Callable, m: int | None = None):
    """(per-element ||E - v_h||_K^2 + ||curl E - curl v_h||_K^2 [T], their total)
    for the Nedelec field v_h with edge values v. On an element
    v_h = sum_k s_k v_k B_K^-T eta^_k and curl v_h = sum_k s_k v_k curl^eta^_k / det B_K
    (2D, scalar) or B_K curl^eta^_k / det B_K (3D): the Piola maps of Section 2.2."""
    dim = elems.shape[1] - 1
    m = DEFAULT_M[dim] if m is None else m
    B, b, det = affine_transformations(nodes, elems)
    BmT = np.swapaxes(np.linalg.inv(B), 1, 2)
    S = element_signs(topo, "ned").astype(np.float64)
    D = element_dofs(topo, "ned")
    ve = np.asarray(v)[D] * S                                       # [T, n]
    cref = ref.curl_basis("ned", dim)
    if dim == 2:
        curl_v = (ve @ cref) / det                                  # [T]
    else:
        curl_v = np.einsum("tij,kj,tk->ti", B, cref, ve) / det[:, None]   # [T, 3]
    xq, wq = ref.quadrature(dim, m)
    per = np.zeros(elems.shape[0])
    for i in range(len(wq)):
        X = np.einsum("tij,j->ti", B, xq[i]) + b
        vh = np.einsum("tki,tk->ti", _ned_basis_at(BmT, xq[i], dim), ve)
        d = E(X) - vh
        c = np.asarray(curlE(X)) - curl_v
        cc = c * c if c.ndim == 1 else np.sum(c * c, axis=1)
        per += wq[i] * np.abs(det) * (np.sum(d * d, axis=1) + cc)
    return per, float(np.sum(per))
