"""Pins of the oracle's integration routine (Section 3.1) and of its 2D
eddy-current example (Section 4.2) against what the paper and the mathematics
fix:

* the paper's printed energy errors of the eddy table, to all printed digits
  (tests/golden/paper_eddy_errors.txt, meshes of 128, 256 and 512 cells per
  side);
* the paper's printed curl E (typed here from the example) against the
  oracle's symbolic curl, and the properties the example states: tangential
  continuity of E and vanishing curl E on the diagonal, vanishing curl E on the
  boundary;
* the squared L2 norm of monomials over the unit square and cube (exact
  integrals) on perturbed meshes, and the affine maps sending reference
  vertices to element vertices;
* the load vector of a discrete Nedelec field w_h equals M times its dof vector
  (the integrand is of degree 2, integrated exactly), and the energy error of
  v against w_h is (v - w)^T (K + M) (v - w) exactly.
"""
import math
import os
from itertools import product

import numpy as np
import pytest

import meshgen as mg
import oracle
from oracle import eddy as ed
from oracle import integrate as it
from oracle import reference as R
from oracle.assembly import element_dofs, element_signs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_eddy_errors.txt")


def paper_eddy_table():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        n, T, E, err = line.split()
        rows.append((int(n), int(T), int(E), float(err)))
    return rows


def test_golden_table_sizes_follow_the_meshes():
    """The printed element and edge counts are those of the n x n unit-square
    meshes (T = 2 n^2, E = 3 n^2 + 2 n)."""
    for n, T, E, _ in paper_eddy_table():
        assert T == 2 * n * n and E == 3 * n * n + 2 * n


@pytest.mark.parametrize("n", [128, 256, pytest.param(512, marks=pytest.mark.slow)])
def test_eddy_errors_match_the_paper(n):
    row = [r for r in paper_eddy_table() if r[0] == n][0]
    nodes, elems = mg.unit_square(n)
    out = ed.solve(nodes, elems)
    assert elems.shape[0] == row[1] and out["topo"].n_edges == row[2]
    # the printed value is the error rounded to 7 significant digits
    assert f"{out['error']:.6e}" == f"{row[3]:.6e}", (out["error"], row[3])


def test_curl_matches_the_printed_formula():
    rng = np.random.default_rng(0)
    X = rng.random((4000, 2))
    x1, x2 = X[:, 0], X[:, 1]
    printed = 2 * x2 * (x1 - x2) * (x1 - 1) * (2 * x1 - x2 - 1) * np.cos(x2 * (x1 - x2) ** 2 * (x1 - 1) ** 2)
    printed = printed * (x1 > x2)
    assert np.allclose(ed.exact_curl_E(X), printed, rtol=0, atol=1e-13)


def test_example_properties():
    t = np.linspace(0, 1, 101)
    diag = np.stack([t + 1e-14, t], axis=1)  # just inside Omega_1
    E = ed.exact_E(diag)
    n = np.array([1.0, -1.0]) / np.sqrt(2.0)
    assert np.abs(E[:, 0] * n[1] - E[:, 1] * n[0]).max() < 1e-12   # E x n = 0 on the diagonal
    assert np.abs(ed.exact_curl_E(diag)).max() < 1e-12
    # curl E = 0 on the boundary parts of Omega_1: x2 = 0 and x1 = 1
    b1 = np.stack([t, np.zeros_like(t)], axis=1)
    b2 = np.stack([np.ones_like(t), t], axis=1)
    assert np.abs(ed.exact_curl_E(b1)).max() < 1e-13 and np.abs(ed.exact_curl_E(b2)).max() < 1e-13
    # E = 0 and F = 0 on Omega_2
    X = np.array([[0.2, 0.7], [0.5, 0.9]])
    assert not ed.exact_E(X).any() and not ed.load_F(X).any()


def test_load_F_is_the_strong_operator():
    """F = curl_vec curl E + E by central differences of the symbolic curl."""
    rng = np.random.default_rng(1)
    X = rng.random((200, 2))
    X = X[X[:, 0] > X[:, 1] + 0.05]
    h = 1e-5
    c = ed.exact_curl_E
    dc1 = (c(X + [h, 0]) - c(X - [h, 0])) / (2 * h)
    dc2 = (c(X + [0, h]) - c(X - [0, h])) / (2 * h)
    F = ed.load_F(X)
    E = ed.exact_E(X)
    assert np.allclose(F[:, 0], dc2 + E[:, 0], atol=1e-7)
    assert np.allclose(F[:, 1], -dc1 + E[:, 1], atol=1e-7)


@pytest.mark.parametrize("dim", [2, 3])
def test_norm_L2_of_monomials_is_exact(dim):
    """||x^p||^2 over the unit square / cube for every monomial of degree <= 3
    (the paper's order-6 setting: exact for cubic f)."""
    rng = np.random.default_rng(2)
    if dim == 2:
        nodes, elems = mg.unit_square(5, 4)
        nodes = mg.perturb_interior(nodes, 0.2, 0.25, rng)
    else:
        nodes, elems = mg.kuhn_box(3, 2, 2)
        nodes = mg.perturb_interior(nodes, 1 / 3, 0.2, rng)
    for exps in product(range(4), repeat=dim):
        if sum(exps) > 3:
            continue
        f = lambda X, e=exps: np.prod(X ** np.array(e), axis=1)  # noqa: E731
        per, tot = it.norm_L2_squared(nodes, elems, f)
        exact = math.prod(1.0 / (2 * e + 1) for e in exps)
        assert abs(tot - exact) < 1e-14, (exps, tot, exact)
        assert per.shape == (elems.shape[0],) and (per >= 0).all()
    # and a vector function: |(x1, x2^2)|^2 -> 1/3 + 1/5 on the unit domain
    per, tot = it.norm_L2_squared(nodes, elems, lambda X: np.stack([X[:, 0], X[:, 1] ** 2], 1))
    assert abs(tot - (1 / 3 + 1 / 5)) < 1e-14


def test_affine_maps_send_reference_vertices_to_the_element():
    rng = np.random.default_rng(3)
    nodes, elems = mg.kuhn_box(2, 2, 2)
    nodes = mg.perturb_interior(nodes, 0.5, 0.2, rng)
    B, b, det = it.affine_transformations(nodes, elems)
    for v in range(4):
        X = np.einsum("tij,j->ti", B, R.REF_NODES[3][v]) + b
        assert np.allclose(X, nodes[elems[:, v]], atol=1e-15)
    assert np.allclose(det, np.linalg.det(B))


def _mesh(dim, seed):
    rng = np.random.default_rng(seed)
    if dim == 2:
        nodes, elems = mg.unit_square(6, 5)
        return mg.perturb_interior(nodes, 1 / 6, 0.2, rng), elems, rng
    nodes, elems = mg.kuhn_box(3, 2, 2)
    return mg.perturb_interior(nodes, 1 / 3, 0.2, rng), elems, rng


def _discrete_field(nodes, elems, topo, c):
    """A Nedelec field w_h with edge values c and its curl, as functions of
    points X [T, d] where row t lies in element t (the way the quadrature loops
    call them)."""
    dim = elems.shape[1] - 1
    B, b, det = it.affine_transformations(nodes, elems)
    Binv = np.linalg.inv(B)
    BmT = np.swapaxes(Binv, 1, 2)
    S = element_signs(topo, "ned").astype(float)
    ce = c[element_dofs(topo, "ned")] * S
    cref = R.curl_basis("ned", dim)

    def w(X):
        xr = np.einsum("tij,tj->ti", Binv, X - b)                  # reference coordinates
        vals = np.stack([xr @ P.T + q for P, q in R.basis("ned", dim)], 1)   # [T, n, d]
        return np.einsum("tij,tkj,tk->ti", BmT, vals, ce)

    def curl(X):
        if dim == 2:
            return (ce @ cref) / det
        return np.einsum("tij,kj,tk->ti", B, cref, ce) / det[:, None]
    return w, curl


@pytest.mark.parametrize("dim", [2, 3])
def test_load_vector_of_a_discrete_field_is_M_times_its_dofs(dim):
    nodes, elems, rng = _mesh(dim, 4)
    csr, topo = oracle.assemble(nodes, elems, "ned")
    c = rng.normal(size=topo.n_edges)
    w, _ = _discrete_field(nodes, elems, topo, c)
    f = it.load_vector_ned(nodes, elems, topo, w)
    assert np.allclose(f, csr.scipy("M") @ c, rtol=0, atol=1e-13 * np.abs(f).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_energy_error_against_a_discrete_field_is_the_matrix_norm(dim):
    nodes, elems, rng = _mesh(dim, 5)
    csr, topo = oracle.assemble(nodes, elems, "ned")
    c = rng.normal(size=topo.n_edges)
    d = rng.normal(size=topo.n_edges)
    w, cw = _discrete_field(nodes, elems, topo, c)
    per, err2 = it.hcurl_error_ned(nodes, elems, topo, c + d, w, cw)
    A = csr.scipy("K") + csr.scipy("M")
    assert abs(err2 - d @ (A @ d)) < 1e-12 * (d @ (A @ d))
    assert abs(per.sum() - err2) < 1e-15 * err2
    _, err0 = it.hcurl_error_ned(nodes, elems, topo, c, w, cw)
    assert err0 < 1e-26
