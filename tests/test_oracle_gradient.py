"""Pins of the oracle's gradient of L = u^T (K(a) + M(b)) u.

* complex-step vertex derivatives against central finite differences of the
  full oracle assembly (step 1e-6);
* exact identities: sum_K a_K dL/da_K = L_K (linearity in a), translation
  invariance sum_v dL/dx_v = 0, rotation invariance sum_v x_v x dL/dx_v = 0,
  and Euler's relation for the scaling degree of each matrix:
  sum_v x_v . dL/dx_v = -L_K + L_M (Ned 3D), -3 L_K - L_M (RT 3D), -2 L_K (2D).
"""
import numpy as np
import pytest

import meshgen as mg
from oracle import assemble
from oracle.assembly import element_dofs
from oracle.gradient import (grad_coefficients, grad_nodes, loss, positions,
                             quadratic_weights)


def setup_case(case, seed=0):
    rng = np.random.default_rng(seed)
    if case.endswith("3"):
        nodes, elems = mg.kuhn_box(2, 2, 1)
        nodes = mg.perturb_interior(nodes, 0.5, 0.2, rng) + rng.normal(size=3)
    else:
        nodes, elems = mg.unit_square(3)
        nodes = mg.perturb_interior(nodes, 1 / 3, 0.2, rng) + rng.normal(size=2)
    kind = case[:-1]
    T = elems.shape[0]
    a = rng.uniform(0.5, 2, T)
    b = rng.uniform(0.5, 2, T)
    csr, topo = assemble(nodes, elems, kind, a=a, b=b)
    u = rng.normal(size=csr.n_rows)
    return nodes, elems, kind, a, b, csr, topo, u


def split_loss(csr, u):
    w = quadratic_weights(csr, u)
    return float(np.dot(w, csr.Kv)), float(np.dot(w, csr.Mv))


@pytest.mark.parametrize("case", ["ned3", "rt3", "ned2", "rt2"])
def test_complex_step_matches_central_differences(case):
    nodes, elems, kind, a, b, csr, topo, u = setup_case(case, 1)
    w = quadratic_weights(csr, u)
    pos = positions(csr, element_dofs(topo, kind))
    g = grad_nodes(nodes, elems, kind, topo, pos, w, w, a, b)
    rng = np.random.default_rng(2)
    h = 1e-6
    for _ in range(6):
        v = rng.integers(nodes.shape[0])
        c = rng.integers(nodes.shape[1])
        xp = nodes.copy()
        xm = nodes.copy()
        xp[v, c] += h
        xm[v, c] -= h
        Lp = loss(assemble(xp, elems, kind, a=a, b=b, topo=topo)[0], u)
        Lm = loss(assemble(xm, elems, kind, a=a, b=b, topo=topo)[0], u)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[v, c]) < 1e-6 * max(1.0, abs(g).max()), (v, c, fd, g[v, c])


@pytest.mark.parametrize("case", ["ned3", "rt3", "ned2", "rt2"])
def test_gradient_identities(case):
    nodes, elems, kind, a, b, csr, topo, u = setup_case(case, 3)
    w = quadratic_weights(csr, u)
    pos = positions(csr, element_dofs(topo, kind))
    ga, gb = grad_coefficients(nodes, elems, kind, topo, pos, w, w)
    g = grad_nodes(nodes, elems, kind, topo, pos, w, w, a, b)
    LK, LM = split_loss(csr, u)
    scale = abs(LK) + abs(LM)
    assert abs(np.dot(a, ga) - LK) < 1e-12 * scale
    assert abs(np.dot(b, gb) - LM) < 1e-12 * scale
    gscale = np.abs(g).max() * np.abs(nodes).max()
    assert np.abs(g.sum(axis=0)).max() < 1e-12 * gscale * 10
    if nodes.shape[1] == 3:
        rot = np.cross(nodes, g).sum(axis=0)
    else:
        rot = np.sum(nodes[:, 0] * g[:, 1] - nodes[:, 1] * g[:, 0])
    assert np.abs(rot).max() < 1e-12 * gscale * 10
    # Euler relation about the centroid (translation invariance lets us shift)
    xc = nodes - nodes.mean(axis=0)
    euler = np.sum(xc * g)
    expect = {"ned3": -LK + LM, "rt3": -3 * LK - LM, "ned2": -2 * LK, "rt2": -2 * LK}[case]
    assert abs(euler - expect) < 1e-11 * scale
