"""Pins of the oracle's global matrices against identities the mathematics fixes.

* textbook closed forms on single elements of arbitrary shape and orientation:
  Whitney 1-forms (Nedelec) and (x - x_p)/(d|K|) fields (Raviart-Thomas),
  integrated exactly with int lambda_a lambda_b = |K| (1 + delta_ab)/((d+1)(d+2));
* discrete de Rham sequence: K^Ned G = 0, K^RT C = 0, K^Ned(a) = C^T M^RT(a) C;
* interpolated constant fields: u^T M(b) u = sum_K b_K |K| |c|^2, u^T K(a) u = 0;
* 2D: the Raviart-Thomas and Nedelec matrices coincide;
* spectra: M symmetric positive definite, rank K^Ned3D = E - V + 1,
  rank K^RT3D = T, rank K^2D = T on contractible meshes;
* CSR structure: nnz = E + 6F + 6T (Ned 3D), F + 12T (RT 3D), E + 6T (2D);
* row subsets equal the corresponding rows of the full assembly.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import meshgen as mg
from oracle import assemble, assemble_rows, build_topology
from oracle.assembly import local_matrices


def perturbed_kuhn(nx, ny, nz, seed=0, delta=0.2):
    nodes, elems = mg.kuhn_box(nx, ny, nz)
    rng = np.random.default_rng(seed)
    nodes = mg.perturb_interior(nodes, 1.0 / max(nx, ny, nz), delta, rng)
    return nodes, elems, rng


def perturbed_square(n, seed=0, delta=0.2):
    nodes, elems = mg.unit_square(n)
    rng = np.random.default_rng(seed)
    return mg.perturb_interior(nodes, 1.0 / n, delta, rng), elems, rng


def relabel(nodes, elems, seed):
    rng = np.random.default_rng(seed)
    perm = rng.permutation(nodes.shape[0])
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    e2 = inv[elems]
    for t in range(e2.shape[0]):
        e2[t] = e2[t][rng.permutation(e2.shape[1])]
    return nodes[perm], e2.astype(np.int32)


# ---------------------------------------------------------------- closed forms
def _bary_gradients(X):
    """Gradients of the barycentric coordinates of simplex X [d+1, d] -> [d+1, d]."""
    d = X.shape[1]
    A = np.vstack([X.T, np.ones(d + 1)])       # lambda = A^-1 [x; 1]
    Ainv = np.linalg.inv(A)
    return Ainv[:, :d]


def _simplex_volume(X):
    d = X.shape[1]
    return abs(np.linalg.det((X[1:] - X[:1]).T)) / (1 if d == 1 else (2 if d == 2 else 6))


def _lam_mass(d):
    L = np.full((d + 1, d + 1), 1.0)
    L += np.eye(d + 1)
    return L / ((d + 1) * (d + 2))             # int lambda_a lambda_b / |K|


@pytest.mark.parametrize("seed", range(4))
def test_ned3d_local_matrices_equal_whitney_closed_form(seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(4, 3))
    elems = np.array([rng.permutation(4) + 10 * seed])
    nodes = np.zeros((elems.max() + 1, 3))
    nodes[elems[0]] = X
    topo = build_topology(elems, nodes.shape[0])
    K, M = local_matrices(nodes, elems, "ned", topo.signs_e)
    # global Nedelec function of edge {p, q}: direction from the larger to the
    # smaller global node index: w = l_hi grad l_lo - l_lo grad l_hi
    Xe = nodes[elems[0]]
    G = _bary_gradients(Xe)
    vol = _simplex_volume(Xe)
    L = _lam_mass(3) * vol
    from oracle.reference import LOCAL_EDGES
    ed = []
    for s, t in LOCAL_EDGES[3]:
        gs, gt = elems[0, s], elems[0, t]
        ed.append((s, t) if gs > gt else (t, s))   # (hi, lo) local indices
    Mw = np.zeros((6, 6))
    Kw = np.zeros((6, 6))
    for k, (i, j) in enumerate(ed):
        for l, (m, n) in enumerate(ed):
            g = G @ G.T
            Mw[k, l] = g[j, n] * L[i, m] - g[j, m] * L[i, n] - g[i, n] * L[j, m] + g[i, m] * L[j, n]
            Kw[k, l] = vol * 4 * np.dot(np.cross(G[i], G[j]), np.cross(G[m], G[n]))
    assert np.allclose(M[0], Mw, rtol=1e-12, atol=1e-12 * np.abs(Mw).max())
    assert np.allclose(K[0], Kw, rtol=1e-12, atol=1e-12 * np.abs(Kw).max())


@pytest.mark.parametrize("seed", range(4))
def test_rt3d_local_matrices_equal_closed_form(seed):
    rng = np.random.default_rng(100 + seed)
    X = rng.normal(size=(4, 3))
    elems = np.array([rng.permutation(4)])
    nodes = np.zeros((4, 3))
    nodes[elems[0]] = X
    topo = build_topology(elems, 4)
    K, M = local_matrices(nodes, elems, "rt", topo.signs_f)
    Xe = nodes[elems[0]]
    vol = _simplex_volume(Xe)
    L = _lam_mass(3) * vol
    from oracle.reference import LOCAL_FACES, FACE_OPPOSITE
    centroid = Xe.mean(axis=0)
    coef = []
    opp = []
    for k, f in enumerate(LOCAL_FACES):
        g = sorted(elems[0, list(f)])
        xa, xb, xc = nodes[g[0]], nodes[g[1]], nodes[g[2]]
        nf = np.cross(xb - xa, xc - xa)
        sigma = np.sign(np.dot(nf, xa - centroid))   # +1 if n_f points outwards
        p = FACE_OPPOSITE[k]
        coef.append(0.5 * sigma / (3 * vol))         # flux 1/2 along n_f
        opp.append(p)
    Mc = np.zeros((4, 4))
    Kc = np.zeros((4, 4))
    for k in range(4):
        for l in range(4):
            Dk = Xe - Xe[opp[k]]
            Dl = Xe - Xe[opp[l]]
            Mc[k, l] = coef[k] * coef[l] * np.sum(L * (Dk @ Dl.T))
            Kc[k, l] = coef[k] * coef[l] * 9 * vol     # div (x - x_p) = 3
    assert np.allclose(M[0], Mc, rtol=1e-12, atol=1e-13 * np.abs(Mc).max())
    assert np.allclose(K[0], Kc, rtol=1e-12, atol=1e-13 * np.abs(Kc).max())


# ---------------------------------------------------------------- global identities
def _gradient_matrix(topo):
    E = topo.n_edges
    lo, hi = topo.edges2nodes[:, 0], topo.edges2nodes[:, 1]
    r = np.concatenate([np.arange(E), np.arange(E)])
    c = np.concatenate([lo, hi])
    v = np.concatenate([np.ones(E), -np.ones(E)])
    return sp.csr_matrix((v, (r, c)), shape=(E, topo.n_nodes))


def _curl_matrix(topo):
    eid = {tuple(e): i for i, e in enumerate(topo.edges2nodes.tolist())}
    rows, cols, vals = [], [], []
    for f, (a, b, c) in enumerate(topo.faces2nodes.tolist()):
        for (p, q), v in (((a, b), -2.0), ((b, c), -2.0), ((a, c), 2.0)):
            rows.append(f)
            cols.append(eid[(p, q)])
            vals.append(v)
    return sp.csr_matrix((vals, (rows, cols)), shape=(topo.n_faces, topo.n_edges))


@pytest.mark.parametrize("shape", [(2, 2, 2), (3, 2, 1)])
def test_de_rham_identities_3d(shape):
    nodes, elems, rng = perturbed_kuhn(*shape, seed=1)
    nodes, elems = relabel(nodes, elems, 3)
    a = rng.uniform(0.5, 2, elems.shape[0])
    ned, topo = assemble(nodes, elems, "ned", a=a)
    rt, _ = assemble(nodes, elems, "rt", a=a, b=a, topo=topo)
    Kn = ned.scipy("K")
    G = _gradient_matrix(topo)
    C = _curl_matrix(topo)
    scale = abs(Kn).max()
    assert abs(Kn @ G).max() < 1e-13 * scale * 10
    assert abs(rt.scipy("K") @ C).max() < 1e-13 * abs(rt.scipy("K")).max() * 10
    diff = Kn - C.T @ rt.scipy("M") @ C
    assert abs(diff).max() < 1e-13 * scale * 10


def test_gradient_in_kernel_2d():
    nodes, elems, rng = perturbed_square(4, seed=2)
    nodes, elems = relabel(nodes, elems, 4)
    ned, topo = assemble(nodes, elems, "ned", a=rng.uniform(0.5, 2, elems.shape[0]))
    G = _gradient_matrix(topo)
    assert abs(ned.scipy("K") @ G).max() < 1e-12


@pytest.mark.parametrize("case", ["ned3", "rt3", "ned2", "rt2"])
def test_constant_field_identity(case):
    if case.endswith("3"):
        nodes, elems, rng = perturbed_kuhn(3, 2, 2, seed=5)
    else:
        nodes, elems, rng = perturbed_square(5, seed=5)
    nodes, elems = relabel(nodes, elems, 9)
    kind = case[:-1]
    T = elems.shape[0]
    a = rng.uniform(0.5, 2, T)
    b = rng.lognormal(0, 0.5, T)
    csr, topo = assemble(nodes, elems, kind, a=a, b=b)
    d = nodes.shape[1]
    c = rng.normal(size=d)
    if kind == "ned" or d == 2:
        lo, hi = topo.edges2nodes[:, 0], topo.edges2nodes[:, 1]
        u = (nodes[lo] - nodes[hi]) @ c
    else:
        fa, fb, fc = topo.faces2nodes.T
        u = np.cross(nodes[fb] - nodes[fa], nodes[fc] - nodes[fa]) @ c
    X = nodes[elems]
    vol = np.abs(np.linalg.det(np.transpose(X[:, 1:] - X[:, :1], (0, 2, 1)))) / (2 if d == 2 else 6)
    expect = np.sum(b * vol) * np.dot(c, c)
    M = csr.scipy("M")
    K = csr.scipy("K")
    assert abs(u @ (M @ u) - expect) < 1e-13 * expect * 10
    assert abs(u @ (K @ u)) < 1e-12 * abs(K).max() * np.dot(u, u)


def test_2d_rt_equals_ned():
    nodes, elems, rng = perturbed_square(6, seed=8)
    nodes, elems = relabel(nodes, elems, 2)
    a = rng.uniform(0.5, 2, elems.shape[0])
    n, topo = assemble(nodes, elems, "ned", a=a, b=a)
    r, _ = assemble(nodes, elems, "rt", a=a, b=a, topo=topo)
    assert np.array_equal(n.colind, r.colind) and np.array_equal(n.rowptr, r.rowptr)
    assert np.allclose(n.Kv, r.Kv, rtol=1e-13, atol=1e-13 * abs(n.Kv).max())
    assert np.allclose(n.Mv, r.Mv, rtol=1e-13, atol=1e-13 * abs(n.Mv).max())


@pytest.mark.parametrize("case", ["ned3", "rt3", "ned2"])
def test_spectra_and_nnz(case):
    if case.endswith("3"):
        nodes, elems, rng = perturbed_kuhn(2, 2, 1, seed=6)
    else:
        nodes, elems, rng = perturbed_square(4, seed=6)
    kind = case[:-1]
    csr, topo = assemble(nodes, elems, kind)
    V, T, E, F = nodes.shape[0], elems.shape[0], topo.n_edges, topo.n_faces
    M = csr.scipy("M").toarray()
    K = csr.scipy("K").toarray()
    assert np.array_equal(M, M.T) and np.array_equal(K, K.T)
    assert np.linalg.eigvalsh(M).min() > 0
    rank = np.linalg.matrix_rank(K, tol=1e-10 * np.abs(K).max())
    if case == "ned3":
        assert rank == E - V + 1
        assert csr.nnz == E + 6 * F + 6 * T
    elif case == "rt3":
        assert rank == T
        assert csr.nnz == F + 12 * T
    else:
        assert rank == T
        assert csr.nnz == E + 6 * T


def test_row_subset_equals_full_rows():
    nodes, elems, rng = perturbed_kuhn(2, 3, 2, seed=4)
    a = rng.uniform(0.5, 2, elems.shape[0])
    b = rng.uniform(0.5, 2, elems.shape[0])
    for kind in ("ned", "rt"):
        full, topo = assemble(nodes, elems, kind, a=a, b=b)
        rows = rng.choice(full.n_rows, 15, replace=False)
        sub, _ = assemble_rows(nodes, elems, kind, rows, a=a, b=b, topo=topo)
        for r, (cols, kv, mv) in sub.items():
            s, e = full.rowptr[r], full.rowptr[r + 1]
            assert np.array_equal(cols, full.colind[s:e])
            assert np.allclose(kv, full.Kv[s:e], rtol=1e-14, atol=1e-14)
            assert np.allclose(mv, full.Mv[s:e], rtol=1e-14, atol=1e-14)
