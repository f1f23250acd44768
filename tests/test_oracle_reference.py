"""Pins of the oracle's reference-element layer against what the paper fixes.

* quadrature: exact monomial integrals over the reference simplex
  (int x^a y^b z^c = a! b! c! / (a+b+c+d)!);
* reference bases: the degree-of-freedom definitions of Section 2.1 (normal
  flux through edges/faces) and Section 2.2 (tangential line integrals), which
  the printed bases must satisfy (3D Raviart-Thomas gives 1/2 on the diagonal:
  the printed 3D basis has flux 1/2 through its face);
* curls: Stokes' theorem on every reference face (line integrals of the basis);
* reference-element matrices: exact symbolic integration (sympy) of the
  printed basis against the oracle's quadrature.
"""
import math
from itertools import product

import numpy as np
import pytest
import sympy as sp

from oracle import reference as R
from oracle.assembly import local_matrices_from_B


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("m", [3, 4])
def test_quadrature_exact_on_monomials(dim, m):
    """The m-point conical rule is exact to total degree 2m - dim (3 points per
    direction, the oracle's rule: degree 4 in 2D, 3 in 3D)."""
    x, w = R.quadrature(dim, m)
    deg = 2 * m - dim
    assert abs(w.sum() - R.REF_VOLUME[dim]) < 1e-15
    for exps in product(range(deg + 1), repeat=dim):
        if sum(exps) > deg:
            continue
        exact = math.prod(math.factorial(e) for e in exps) / math.factorial(sum(exps) + dim)
        val = np.sum(w * np.prod(x ** np.array(exps), axis=1))
        assert abs(val - exact) < 1e-15, (exps, val, exact)
    # and not exact one degree higher (the rule is the one described)
    exps = (deg + 1,) + (0,) * (dim - 1)
    exact = math.factorial(deg + 1) / math.factorial(deg + 1 + dim)
    assert abs(np.sum(w * x[:, 0] ** (deg + 1)) - exact) > 1e-12


def _line_integral(f, xs, xt, m=5):
    t, w = R.gauss_legendre_01(m)
    pts = xs[None, :] + t[:, None] * (xt - xs)[None, :]
    return np.sum(w * f(pts)) * np.linalg.norm(xt - xs)


def _edge_dofs(kind, dim):
    """alpha_i(eta_j): tangential (Ned) or normal (RT 2D) line integrals, Figure 1."""
    nodes = R.REF_NODES[dim]
    nb = R.n_local(kind, dim)
    A = np.zeros((nb, nb))
    for i, (s, t) in enumerate(R.LOCAL_EDGES[dim]):
        xs, xt = nodes[s], nodes[t]
        tau = (xt - xs) / np.linalg.norm(xt - xs)
        if kind == "ned":
            direction = tau
        else:
            # 2D outward normal of edge i (the edge opposite node i)
            nvec = np.array([tau[1], -tau[0]])
            mid = 0.5 * (xs + xt)
            if np.dot(nvec, mid - nodes[i]) < 0:
                nvec = -nvec
            direction = nvec
        for j in range(nb):
            f = lambda p, j=j: R.eval_basis(kind, dim, p)[:, j, :] @ direction
            A[i, j] = _line_integral(f, xs, xt)
    return A


@pytest.mark.parametrize("kind,dim", [("ned", 2), ("ned", 3), ("rt", 2)])
def test_edge_dofs_are_kronecker(kind, dim):
    A = _edge_dofs(kind, dim)
    assert np.allclose(A, np.eye(A.shape[0]), atol=1e-14), A


def _face_quadrature(xa, xb, xc):
    p, w = R.quadrature(2, 4)
    pts = xa[None] + p[:, :1] * (xb - xa)[None] + p[:, 1:2] * (xc - xa)[None]
    area2 = np.linalg.norm(np.cross(xb - xa, xc - xa))
    return pts, w * area2  # weights sum to the face area


def test_rt3d_face_fluxes_are_half_kronecker():
    nodes = R.REF_NODES[3]
    A = np.zeros((4, 4))
    centroid = nodes.mean(axis=0)
    for i, f in enumerate(R.LOCAL_FACES):
        xa, xb, xc = nodes[list(f)]
        n = np.cross(xb - xa, xc - xa)
        n /= np.linalg.norm(n)
        if np.dot(n, xa - centroid) < 0:
            n = -n
        pts, w = _face_quadrature(xa, xb, xc)
        vals = R.eval_basis("rt", 3, pts)
        for j in range(4):
            A[i, j] = np.sum(w * (vals[:, j, :] @ n))
    # Face i of Figure 1 is opposite node 4-i; the printed basis has flux 1/2.
    assert np.allclose(A, 0.5 * np.eye(4), atol=1e-14), A


def test_ned3d_curl_satisfies_stokes_on_every_face():
    nodes = R.REF_NODES[3]
    curls = R.curl_basis("ned", 3)
    for f in R.LOCAL_FACES:
        xa, xb, xc = nodes[list(f)]
        nvec = np.cross(xb - xa, xc - xa)           # |nvec| = 2 * area
        for j in range(6):
            flux = 0.5 * np.dot(curls[j], nvec)
            circ = 0.0
            for s, t in ((xa, xb), (xb, xc), (xc, xa)):
                tau = (t - s) / np.linalg.norm(t - s)
                circ += _line_integral(lambda p: R.eval_basis("ned", 3, p)[:, j, :] @ tau, s, t)
            assert abs(flux - circ) < 1e-14


def test_ned2d_curl_and_rt_div_by_divergence_theorem():
    nodes2 = R.REF_NODES[2]
    c2 = R.curl_basis("ned", 2)
    for j in range(3):
        circ = 0.0
        for s, t in ((0, 1), (1, 2), (2, 0)):
            xs, xt = nodes2[s], nodes2[t]
            tau = (xt - xs) / np.linalg.norm(xt - xs)
            circ += _line_integral(lambda p: R.eval_basis("ned", 2, p)[:, j, :] @ tau, xs, xt)
        assert abs(c2[j] * 0.5 - circ) < 1e-14
    # div: total outward flux = div * |K|
    for dim in (2, 3):
        A = _edge_dofs("rt", 2) if dim == 2 else None
        dv = R.div_basis("rt", dim)
        if dim == 2:
            assert np.allclose(A.sum(axis=0), dv * R.REF_VOLUME[2])
        else:
            assert np.allclose(0.5 * np.ones(4), dv * R.REF_VOLUME[3])


def _sympy_basis(kind, dim):
    x = sp.symbols("x1:%d" % (dim + 1))
    out = []
    for P, q in R.basis(kind, dim):
        out.append([sum(sp.Rational(int(P[i, j])) * x[j] for j in range(dim)) + sp.Rational(int(q[i]))
                    for i in range(dim)])
    return x, out


def _sympy_simplex_integral(expr, x):
    if len(x) == 2:
        return sp.integrate(sp.integrate(expr, (x[1], 0, 1 - x[0])), (x[0], 0, 1))
    return sp.integrate(sp.integrate(sp.integrate(expr, (x[2], 0, 1 - x[0] - x[1])),
                                     (x[1], 0, 1 - x[0])), (x[0], 0, 1))


@pytest.mark.parametrize("kind,dim", [("rt", 2), ("ned", 2), ("rt", 3), ("ned", 3)])
def test_reference_matrices_match_exact_symbolic_integrals(kind, dim):
    x, bas = _sympy_basis(kind, dim)
    n = len(bas)
    Mex = np.zeros((n, n))
    Kex = np.zeros((n, n))
    for k in range(n):
        for l in range(n):
            Mex[k, l] = float(_sympy_simplex_integral(sum(bas[k][i] * bas[l][i] for i in range(dim)), x))
            if kind == "rt":
                dk = sum(sp.diff(bas[k][i], x[i]) for i in range(dim))
                dl = sum(sp.diff(bas[l][i], x[i]) for i in range(dim))
                Kex[k, l] = float(_sympy_simplex_integral(dk * dl, x))
            elif dim == 2:
                ck = sp.diff(bas[k][1], x[0]) - sp.diff(bas[k][0], x[1])
                cl = sp.diff(bas[l][1], x[0]) - sp.diff(bas[l][0], x[1])
                Kex[k, l] = float(_sympy_simplex_integral(ck * cl, x))
            else:
                def curl(v):
                    return [sp.diff(v[2], x[1]) - sp.diff(v[1], x[2]),
                            sp.diff(v[0], x[2]) - sp.diff(v[2], x[0]),
                            sp.diff(v[1], x[0]) - sp.diff(v[0], x[1])]
                ck, cl = curl(bas[k]), curl(bas[l])
                Kex[k, l] = float(_sympy_simplex_integral(sum(ck[i] * cl[i] for i in range(3)), x))
    K, M = local_matrices_from_B(np.eye(dim)[None], kind, np.ones((1, n), dtype=np.int8))
    assert np.allclose(K[0], Kex, rtol=0, atol=1e-15)
    assert np.allclose(M[0], Mex, rtol=0, atol=1e-15)
