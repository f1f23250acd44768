"""The 2D eddy-current example of Section 4.2 (oracle; test infrastructure).

Problem (Section 4.2): curl_vec(mu^-1 curl E) + kappa E = F in the unit square,
with mu = kappa = 1 and the natural condition mu^-1 curl E = 0 on the whole
boundary (Gamma_D is empty). Weak form: find E in H(curl) with
    int mu^-1 curl E curl w + int kappa E . w = int F . w   for all w.

The exact solution of the example is the printed field E on
Omega_1 = {x1 > x2} and E = 0 on Omega_2; F is formed from it here by symbolic
differentiation (sympy), F = curl_vec curl E + E on each part, where for a
scalar c, curl_vec c = (dc/dx2, -dc/dx1) and for a field v,
curl v = dv2/dx1 - dv1/dx2 (the 2D curls of Section 2).

Discretisation with 2D lowest-order Nedelec elements: K v + M v = f with K, M
from ``assembly.assemble`` (a = 1/mu = 1, b = kappa = 1) and the load vector
f_i = int F . eta_i, eta_i the sign-adjusted covariant Piola image
s_k B_K^-T eta^_k of the reference basis on each element (Section 2.2). The
load integrals and the error integrals use the quadrature of
``integrate`` (the mesh must follow the diagonal x1 = x2, as the unit-square
meshes of ``meshgen`` do, so that every element lies in one part and its
quadrature points are interior to it). The linear system is solved directly
(scipy's sparse LU).

The reported quantity is the energy error of the eddy table,
sqrt(||E - v||^2 + ||curl(E - v)||^2), with curl v = s_k v_k curl^eta^_k / det B_K
on each element (the 2D covariant Piola map scales the curl by 1/det B_K).
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

from .assembly import assemble
from .integrate import DEFAULT_M, hcurl_error_ned, load_vector_ned


@lru_cache(maxsize=1)
def _exact():
    import sympy as sp
    x1, x2 = sp.symbols("x1 x2", real=True)
    pi = sp.pi
    E1 = sp.sin(2 * pi * x1) + 2 * pi * sp.cos(2 * pi * x1) * (x1 - x2)
    E2 = sp.sin((x1 - x2) ** 2 * (x1 - 1) ** 2 * x2) - sp.sin(2 * pi * x1)
    curl = sp.diff(E2, x1) - sp.diff(E1, x2)
    F1 = sp.diff(curl, x2) + E1
    F2 = -sp.diff(curl, x1) + E2
    fE = sp.lambdify((x1, x2), (E1, E2), "numpy")
    fC = sp.lambdify((x1, x2), curl, "numpy")
    fF = sp.lambdify((x1, x2), (F1, F2), "numpy")
    return fE, fC, fF


def _omega1(X):
    return X[:, 0] > X[:, 1]


def exact_E(X: np.ndarray) -> np.ndarray:
    """E at points X [N,2] -> [N,2] (zero where x1 <= x2)."""
    fE, _, _ = _exact()
    v = np.stack(np.broadcast_arrays(*fE(X[:, 0], X[:, 1])), axis=1).astype(np.float64)
    return v * _omega1(X)[:, None]


def exact_curl_E(X: np.ndarray) -> np.ndarray:
    """curl E at points X [N,2] -> [N]."""
    _, fC, _ = _exact()
    return np.broadcast_to(fC(X[:, 0], X[:, 1]), (X.shape[0],)).astype(np.float64) * _omega1(X)


def load_F(X: np.ndarray) -> np.ndarray:
    """F = curl_vec curl E + E at points X [N,2] -> [N,2]."""
    _, _, fF = _exact()
    v = np.stack(np.broadcast_arrays(*fF(X[:, 0], X[:, 1])), axis=1).astype(np.float64)
    return v * _omega1(X)[:, None]


def load_vector(nodes, elems, topo, F=load_F, m=None):
    """f_i = int F . eta_i (``integrate.load_vector_ned``) with the example's F."""
    return load_vector_ned(nodes, elems, topo, F, DEFAULT_M[2] if m is None else m)


def hcurl_error(nodes, elems, topo, v, E=exact_E, curlE=exact_curl_E, m=None):
    """(per-element ||E - v||_K^2 + ||curl(E - v)||_K^2 [T], total
    sqrt(||E - v||^2 + ||curl(E - v)||^2)) for the Nedelec field with edge
    values v."""
    per, tot = hcurl_error_ned(nodes, elems, topo, v, E, curlE, DEFAULT_M[2] if m is None else m)
    return per, float(np.sqrt(tot))


def solve(nodes, elems, mu_inv=None, kappa=None, m=None):
    """The whole example on one mesh: assemble K(1/mu) + M(kappa), the load
    vector, a direct solve and the energy error. Returns a dict with the CSR
    matrices, f, v, the per-element error terms and the error."""
    import scipy.sparse.linalg as spla
    csr, topo = assemble(nodes, elems, "ned", a=mu_inv, b=kappa)
    f = load_vector(nodes, elems, topo, m=m)
    A = (csr.scipy("K") + csr.scipy("M")).tocsc()
    v = spla.spsolve(A, f)
    per, err = hcurl_error(nodes, elems, topo, v, m=m)
    return dict(csr=csr, topo=topo, f=f, v=v, per_elem=per, error=err)
