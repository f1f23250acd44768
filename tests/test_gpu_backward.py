"""GPU adjoint (fem_assemble_backward) against the oracle's gradient and against
central finite differences of the GPU forward, for L = u^T (K(a) + M(b)) u.

Tolerance: the adjoint and the complex-step oracle are both exact up to
rounding; they differ by the conditioning of the per-element formulas
(a few hundred ulps of the largest term), so the check is
max |g_gpu - g_oracle| <= 1e-11 max |g_oracle| for each of dL/da, dL/db, dL/dx.
The quadratic-form entry point evaluates the same contraction with weights
formed from u (3D Nedelec: as sums of squares, a different rounding), so it
is held to max |g_quad - g_general| <= 1e-12 max |g_general| as well as to
the oracle.
"""
import numpy as np
import pytest

import meshgen as mg
import oracle
from gpu_util import dev_tensors, relabel, say
from oracle.gradient import grad_coefficients, grad_nodes, positions, quadratic_weights

pytestmark = pytest.mark.gpu

GTOL = 1e-11
QTOL = 1e-12


def weights_on_device(rowptr, colind, u):
    import torch
    rows = torch.repeat_interleave(torch.arange(rowptr.numel() - 1, device=rowptr.device),
                                   torch.diff(rowptr))
    return u[rows] * u[colind.long()]


def make_case(case, seed):
    rng = np.random.default_rng(seed)
    if case.endswith("3"):
        nodes, elems = relabel(*mg.kuhn_box(3, 2, 2), seed)
        nodes = mg.perturb_interior(nodes, 1 / 3, 0.2, rng) + rng.normal(size=3)
    else:
        nodes, elems = relabel(*mg.unit_square(5, 4), seed)
        nodes = mg.perturb_interior(nodes, 0.2, 0.2, rng) + rng.normal(size=2)
    kind = case[:-1]
    a = rng.lognormal(0, 0.5, elems.shape[0])
    b = rng.uniform(0.5, 2, elems.shape[0])
    return nodes, elems, kind, a, b, rng


@pytest.mark.parametrize("case", ["ned3", "rt3", "ned2", "rt2"])
def test_adjoint_matches_oracle(case):
    import torch
    import paper_1409_4618_amd as fem
    nodes, elems, kind, a, b, rng = make_case(case, 11)
    say(f"[gpu] adjoint vs oracle: {case} T={elems.shape[0]}")
    csr, topo = oracle.assemble(nodes, elems, kind, a=a, b=b)
    u = rng.normal(size=csr.n_rows)
    w = quadratic_weights(csr, u)
    pos = positions(csr, oracle.element_dofs(topo, kind))
    ga_o, gb_o = grad_coefficients(nodes, elems, kind, topo, pos, w, w)
    gn_o = grad_nodes(nodes, elems, kind, topo, pos, w, w, a, b)

    tn, te, ta, tb = dev_tensors(nodes, elems, a, b)
    mesh = fem.Mesh(tn, te)
    rowptr, colind = mesh.pattern(kind)
    tu = torch.tensor(u, device=tn.device)
    tw = weights_on_device(rowptr, colind, tu)
    gn, ga, gb = fem.assemble_backward(mesh, kind, tn, ta, tb, tw, tw)
    mesh.status()
    # the quadratic-form entry point: the same contraction from u at each
    # element's dofs
    qn, qa, qb = fem.assemble_backward_quadratic(mesh, kind, tn, ta, tb, tu)
    mesh.status()
    for q, g, nm in ((qa, ga, "a"), (qb, gb, "b"), (qn, gn, "x")):
        err = float((q - g).abs().max()) / float(g.abs().max())
        say(f"    quadratic vs general dL/d{nm}: {err:.2e}")
        assert err <= QTOL, (nm, err)
    for got, ref, nm in ((ga, ga_o, "a"), (gb, gb_o, "b"), (gn, gn_o, "x"),
                         (qa, ga_o, "a (quadratic)"), (qb, gb_o, "b (quadratic)"), (qn, gn_o, "x (quadratic)")):
        got = got.cpu().numpy()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        say(f"    dL/d{nm}: max rel err {err:.2e}")
        assert err <= GTOL, (nm, err)
    # the autograd path gives the same gradients
    tn2 = tn.clone().requires_grad_(True)
    ta2 = ta.clone().requires_grad_(True)
    tb2 = tb.clone().requires_grad_(True)
    K, M = fem.assemble_autograd(mesh, kind, tn2, ta2, tb2)
    L = (tw * K).sum() + (tw * M).sum()
    L.backward()
    assert torch.equal(tn2.grad, gn) and torch.equal(ta2.grad, ga) and torch.equal(tb2.grad, gb)
    # L itself matches the oracle's
    L_o = float(np.dot(w, csr.Kv) + np.dot(w, csr.Mv))
    assert abs(L.item() - L_o) <= 1e-12 * abs(L_o)


@pytest.mark.parametrize("case", ["ned3", "rt3", "ned2"])
def test_adjoint_matches_central_differences(case):
    import torch
    import paper_1409_4618_amd as fem
    nodes, elems, kind, a, b, rng = make_case(case, 5)
    say(f"[gpu] adjoint vs central FD (h=1e-6): {case}")
    tn, te, ta, tb = dev_tensors(nodes, elems, a, b)
    mesh = fem.Mesh(tn, te)
    rowptr, colind = mesh.pattern(kind)
    _, nnz = mesh.pattern_info(kind)
    tu = torch.tensor(rng.normal(size=rowptr.numel() - 1), device=tn.device)
    tw = weights_on_device(rowptr, colind, tu)

    def L(x, av, bv):
        K, M = fem.assemble(mesh, kind, x, av, bv)
        return float(((tw * K).sum() + (tw * M).sum()).item())

    gn, ga, gb = fem.assemble_backward(mesh, kind, tn, ta, tb, tw, tw)
    h = 1e-6
    scale = max(gn.abs().max().item(), 1.0)
    for _ in range(8):
        v = int(rng.integers(nodes.shape[0]))
        c = int(rng.integers(nodes.shape[1]))
        xp = tn.clone()
        xm = tn.clone()
        xp[v, c] += h
        xm[v, c] -= h
        fd = (L(xp, ta, tb) - L(xm, ta, tb)) / (2 * h)
        assert abs(fd - gn[v, c].item()) <= 1e-6 * scale, (v, c, fd, gn[v, c].item())
    for _ in range(4):
        e = int(rng.integers(elems.shape[0]))
        ap = ta.clone()
        am = ta.clone()
        ap[e] += h
        am[e] -= h
        fd = (L(tn, ap, tb) - L(tn, am, tb)) / (2 * h)
        assert abs(fd - ga[e].item()) <= 1e-6 * max(1.0, ga.abs().max().item())


@pytest.mark.parametrize("case", ["ned3", "rt3", "ned2"])
def test_adjoint_separate_and_missing_weights(case):
    """gK and gM independent, then gM absent (NULL: its part is zero), then both
    absent (L = 0, every derivative zero)."""
    import torch
    import paper_1409_4618_amd as fem
    nodes, elems, kind, a, b, rng = make_case(case, 23)
    say(f"[gpu] adjoint with separate / missing weights: {case}")
    csr, topo = oracle.assemble(nodes, elems, kind, a=a, b=b)
    wK = rng.normal(size=csr.nnz)
    wM = rng.normal(size=csr.nnz)
    pos = positions(csr, oracle.element_dofs(topo, kind))
    tn, te, ta, tb = dev_tensors(nodes, elems, a, b)
    mesh = fem.Mesh(tn, te)
    mesh.pattern(kind)
    for wm, tag in ((wM, "gK, gM"), (None, "gK only")):
        wm_o = np.zeros_like(wK) if wm is None else wm
        ga_o, gb_o = grad_coefficients(nodes, elems, kind, topo, pos, wK, wm_o)
        gn_o = grad_nodes(nodes, elems, kind, topo, pos, wK, wm_o, a, b)
        tK = torch.tensor(wK, device=tn.device)
        tM = None if wm is None else torch.tensor(wm, device=tn.device)
        gn, ga, gb = fem.assemble_backward(mesh, kind, tn, ta, tb, tK, tM)
        mesh.status()
        for got, ref, nm in ((ga, ga_o, "a"), (gb, gb_o, "b"), (gn, gn_o, "x")):
            got = got.cpu().numpy()
            denom = max(np.abs(ref).max(), 1e-300)
            err = np.abs(got - ref).max() / denom if np.abs(ref).max() > 0 else np.abs(got).max()
            say(f"    {tag}: dL/d{nm} max rel err {err:.2e}")
            assert err <= GTOL, (tag, nm, err)
    gn, ga, gb = fem.assemble_backward(mesh, kind, tn, ta, tb, None, None)
    mesh.status()
    assert not bool(gn.abs().max() > 0) and not bool(ga.abs().max() > 0) and not bool(gb.abs().max() > 0)


def multi_wg_case(case):
    """Meshes larger than one 256-element adjoint workgroup, with a partial last
    workgroup: Kuhn 5x4x3 (360 tets = 256 + 104), relabelled; a 12x11 square
    with one interior triangle removed (263 triangles = 256 + 7, so the last
    workgroup has an odd number of vertex incidences, 21)."""
    rng = np.random.default_rng(41)
    if case in ("ned3", "rt3"):
        nodes, elems = relabel(*mg.kuhn_box(5, 4, 3), 9)
        nodes = mg.perturb_interior(nodes, 0.2, 0.2, rng)
    else:
        nodes, elems = relabel(*mg.unit_square(12, 11), 9)
        nodes = mg.perturb_interior(nodes, 1 / 12, 0.2, rng)
        elems = np.delete(elems, elems.shape[0] // 2, axis=0)
    kind = case[:-1]
    a = rng.lognormal(0, 0.5, elems.shape[0])
    b = rng.uniform(0.5, 2, elems.shape[0])
    return nodes, elems, kind, a, b, rng


@pytest.mark.parametrize("case", ["ned3", "rt3", "ned2"])
def test_adjoint_several_workgroups(case):
    import torch
    import paper_1409_4618_amd as fem
    nodes, elems, kind, a, b, rng = multi_wg_case(case)
    say(f"[gpu] adjoint over several workgroups: {case} T={elems.shape[0]}")
    csr, topo = oracle.assemble(nodes, elems, kind, a=a, b=b)
    u = rng.normal(size=csr.n_rows)
    w = quadratic_weights(csr, u)
    pos = positions(csr, oracle.element_dofs(topo, kind))
    ga_o, gb_o = grad_coefficients(nodes, elems, kind, topo, pos, w, w)
    gn_o = grad_nodes(nodes, elems, kind, topo, pos, w, w, a, b)
    tn, te, ta, tb = dev_tensors(nodes, elems, a, b)
    mesh = fem.Mesh(tn, te)
    rowptr, colind = mesh.pattern(kind)
    tu = torch.tensor(u, device=tn.device)
    tw = weights_on_device(rowptr, colind, tu)
    gn, ga, gb = fem.assemble_backward(mesh, kind, tn, ta, tb, tw, tw)
    qn, qa, qb = fem.assemble_backward_quadratic(mesh, kind, tn, ta, tb, tu)
    mesh.status()
    for got, ref, nm in ((ga, ga_o, "a"), (gb, gb_o, "b"), (gn, gn_o, "x"),
                         (qa, ga_o, "a (quadratic)"), (qb, gb_o, "b (quadratic)"), (qn, gn_o, "x (quadratic)")):
        got = got.cpu().numpy()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        say(f"    dL/d{nm}: max rel err {err:.2e}")
        assert err <= GTOL, (nm, err)
    # deterministic: a second call is bitwise identical
    gn2, ga2, gb2 = fem.assemble_backward(mesh, kind, tn, ta, tb, tw, tw)
    mesh.status()
    assert torch.equal(gn, gn2) and torch.equal(ga, ga2) and torch.equal(gb, gb2)
