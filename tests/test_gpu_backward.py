"""GPU adjoint (fem_assemble_backward) against the oracle's gradient and against
central finite differences of the GPU forward, for L = u^T (K(a) + M(b)) u.

Tolerance: the adjoint and the complex-step oracle are both exact up to
rounding, so the check is the stated 1e-12 bound on the relative error,
max |g_gpu - g_oracle| <= 1e-12 max |g_oracle| for each of dL/da, dL/db,
dL/dx (measured errors are a few 1e-16 to 1e-15).
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

GTOL = 1e-12
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


def with_unreferenced_nodes(nodes, elems, n_extra, rng):
    """The same mesh with ``n_extra`` nodes that no element references, placed
    at random positions in the node list (ids of the used nodes get gaps, and
    the first and last ids are unused)."""
    V = nodes.shape[0]
    Vn = V + n_extra
    extra = np.sort(rng.choice(np.arange(1, Vn - 1), size=n_extra - 2, replace=False))
    extra = np.concatenate([[0], extra, [Vn - 1]])
    used = np.setdiff1d(np.arange(Vn), extra)
    out = np.empty((Vn, nodes.shape[1]))
    out[used] = nodes
    out[extra] = rng.uniform(-1.0, 2.0, size=(n_extra, nodes.shape[1]))
    return out, used[elems].astype(np.int32), extra


@pytest.mark.parametrize("case", ["ned3", "rt3", "ned2"])
def test_unreferenced_nodes(case):
    """Nodes that no element references: the forward equals the oracle's, and
    dL/dnodes is exactly 0 at those nodes (both adjoint entry points) and
    matches the oracle elsewhere."""
    import torch
    import paper_1409_4618_amd as fem
    from test_gpu_parity import check_against_oracle, run_case
    nodes, elems, kind, a, b, rng = make_case(case, 31)
    nodes, elems, extra = with_unreferenced_nodes(nodes, elems, 7, rng)
    g = run_case(f"unreferenced nodes {case}", nodes, elems, kind, a, b)
    check_against_oracle(g, nodes, elems, kind, a, b)
    csr, topo = oracle.assemble(nodes, elems, kind, a=a, b=b)
    u = rng.normal(size=csr.n_rows)
    w = quadratic_weights(csr, u)
    pos = positions(csr, oracle.element_dofs(topo, kind))
    gn_o = grad_nodes(nodes, elems, kind, topo, pos, w, w, a, b)
    assert not np.any(gn_o[extra])
    tn, te, ta, tb = dev_tensors(nodes, elems, a, b)
    mesh = g["mesh"]
    rowptr, colind = mesh.pattern(kind)
    tu = torch.tensor(u, device=tn.device)
    tw = weights_on_device(rowptr, colind, tu)
    # outputs pre-filled with NaN: every row must be written
    gn = torch.full_like(tn, float("nan"))
    qn = torch.full_like(tn, float("nan"))
    L = fem._lib.lib()
    from paper_1409_4618_amd import _ptr, _stream_ptr, kind_code
    fem._lib.check(L.fem_assemble_backward(mesh.handle, kind_code(kind), _ptr(tn), _ptr(ta), _ptr(tb),
                                           _ptr(tw), _ptr(tw), None, None, _ptr(gn), _stream_ptr()),
                   "fem_assemble_backward")
    fem._lib.check(L.fem_assemble_backward_quadratic(mesh.handle, kind_code(kind), _ptr(tn), _ptr(ta),
                                                     _ptr(tb), _ptr(tu), None, None, _ptr(qn),
                                                     _stream_ptr()), "fem_assemble_backward_quadratic")
    mesh.status()
    for got, nm in ((gn, "general"), (qn, "quadratic")):
        got = got.cpu().numpy()
        assert np.all(got[extra] == 0.0), nm
        err = np.abs(got - gn_o).max() / np.abs(gn_o).max()
        say(f"    {nm}: dL/dx max rel err {err:.2e}; {extra.size} unreferenced nodes exactly 0")
        assert err <= GTOL, (nm, err)


@pytest.mark.parametrize("case", ["ned3", "rt3", "ned2", "rt2"])
def test_quadratic_form_through_autograd(case):
    """fem.assemble_quadratic: K, M equal fem.assemble's bitwise; L equals the
    oracle's u^T (K + M) u; L.backward() gives dL/da, dL/db, dL/dx equal to the
    oracle's gradient (1e-12 of the largest entry) and dL/du = 2 (K + M) u equal
    to the oracle matrices' product. quadratic_form (no assembly) gives the same
    L and gradients bitwise."""
    import torch
    import paper_1409_4618_amd as fem
    nodes, elems, kind, a, b, rng = make_case(case, 13)
    say(f"[gpu] quadratic form through autograd: {case} T={elems.shape[0]}")
    csr, topo = oracle.assemble(nodes, elems, kind, a=a, b=b)
    u = rng.normal(size=csr.n_rows)
    w = quadratic_weights(csr, u)
    pos = positions(csr, oracle.element_dofs(topo, kind))
    ga_o, gb_o = grad_coefficients(nodes, elems, kind, topo, pos, w, w)
    gn_o = grad_nodes(nodes, elems, kind, topo, pos, w, w, a, b)
    L_o = float(np.dot(w, csr.Kv) + np.dot(w, csr.Mv))
    gu_o = 2.0 * (csr.scipy("K") @ u + csr.scipy("M") @ u)
    tn, te, ta, tb = dev_tensors(nodes, elems, a, b)
    mesh = fem.Mesh(tn, te)
    K0, M0 = fem.assemble(mesh, kind, tn, ta, tb)
    tu = torch.tensor(u, device=tn.device)
    leaves = [t.clone().requires_grad_(True) for t in (tn, ta, tb, tu)]
    K, M, L = fem.assemble_quadratic(mesh, kind, *leaves)
    assert not K.requires_grad and not M.requires_grad
    assert torch.equal(K, K0) and torch.equal(M, M0)
    eL = abs(L.item() - L_o) / abs(L_o)
    say(f"    L rel err {eL:.2e}")
    assert eL <= 1e-12
    L.backward()
    mesh.status()
    for got, ref, nm in ((leaves[1].grad, ga_o, "a"), (leaves[2].grad, gb_o, "b"), (leaves[0].grad, gn_o, "x"),
                         (leaves[3].grad, gu_o, "u")):
        got = got.cpu().numpy()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        say(f"    dL/d{nm}: max rel err {err:.2e}")
        assert err <= GTOL, (nm, err)
    # the same through quadratic_form, which assembles nothing in its forward;
    # an upstream factor of 3 scales every gradient
    leaves2 = [t.clone().requires_grad_(True) for t in (tn, ta, tb, tu)]
    L2 = fem.quadratic_form(mesh, kind, *leaves2)
    assert torch.equal(L2, L.detach())
    (3.0 * L2).backward()
    for g1, g2 in zip(leaves, leaves2):
        assert torch.equal(g2.grad, 3.0 * g1.grad)


@pytest.mark.parametrize("case", ["ned3", "rt3", "ned2", "rt2"])
def test_quadratic_value_adjoint_in_one_pass(case):
    """fem_quadratic_value_adjoint (L with its adjoint, the forward of the
    autograd functions when an input needs a gradient): the derivatives are
    bitwise those of fem_assemble_backward_quadratic (the same kernel), L is
    within 1e-14 of fem_quadratic_value's and 1e-12 of the oracle's, on
    meshes of several workgroups; any subset of the derivatives may be asked
    for; without gradients the autograd forward takes fem_quadratic_value."""
    import torch
    import paper_1409_4618_amd as fem
    rng = np.random.default_rng(29)
    if case.endswith("3"):
        nodes, elems = relabel(*mg.kuhn_box(6, 5, 4), 29)
        nodes = mg.perturb_interior(nodes, 1 / 6, 0.2, rng)
    else:
        nodes, elems = relabel(*mg.unit_square(17, 13), 29)
        nodes = mg.perturb_interior(nodes, 1 / 17, 0.2, rng)
    kind = case[:-1]
    a = rng.lognormal(0, 0.5, elems.shape[0])
    b = rng.uniform(0.5, 2, elems.shape[0])
    say(f"[gpu] quadratic value + adjoint in one pass: {case} T={elems.shape[0]}")
    csr, _ = oracle.assemble(nodes, elems, kind, a=a, b=b)
    u = rng.normal(size=csr.n_rows)
    w = quadratic_weights(csr, u)
    L_o = float(np.dot(w, csr.Kv) + np.dot(w, csr.Mv))
    tn, te, ta, tb = dev_tensors(nodes, elems, a, b)
    mesh = fem.Mesh(tn, te)
    tu = torch.tensor(u, device=tn.device)
    L, gn, ga, gb = fem.quadratic_value_adjoint(mesh, kind, tn, ta, tb, tu)
    gn2, ga2, gb2 = fem.assemble_backward_quadratic(mesh, kind, tn, ta, tb, tu)
    L2 = fem.quadratic_value(mesh, kind, tn, ta, tb, tu)
    mesh.status()
    assert torch.equal(gn, gn2) and torch.equal(ga, ga2) and torch.equal(gb, gb2)
    eL = abs(L.item() - L_o) / abs(L_o)
    say(f"    L rel err {eL:.2e}, against fem_quadratic_value {abs(L.item() - L2.item()) / abs(L2.item()):.1e}")
    assert eL <= 1e-12 and abs(L.item() - L2.item()) <= 1e-14 * abs(L2.item())
    for need in ((True, False, False), (False, True, False), (False, False, True)):
        Lp, gnp, gap, gbp = fem.quadratic_value_adjoint(mesh, kind, tn, ta, tb, tu, need_a=need[0], need_b=need[1],
                                                        need_nodes=need[2])
        mesh.status()
        assert torch.equal(Lp, L)
        for got, ref, want in ((gap, ga, need[0]), (gbp, gb, need[1]), (gnp, gn, need[2])):
            assert (got is None) == (not want)
            if want:
                assert torch.equal(got, ref)
    # no input needs a gradient: the forward computes the value only
    _, _, L3 = fem.assemble_quadratic(mesh, kind, tn, ta, tb, tu)
    assert torch.equal(L3, L2)


@pytest.mark.parametrize("case", ["ned3", "rt3", "ned2"])
def test_assemble_is_differentiable(case):
    """fem.assemble with inputs that require grad routes through the adjoint:
    the gradients of sum(gK K + gM M) equal fem_assemble_backward's bitwise and
    the oracle's within 1e-12."""
    import torch
    import paper_1409_4618_amd as fem
    nodes, elems, kind, a, b, rng = make_case(case, 17)
    say(f"[gpu] differentiable fem.assemble: {case}")
    csr, topo = oracle.assemble(nodes, elems, kind, a=a, b=b)
    wK = rng.normal(size=csr.nnz)
    wM = rng.normal(size=csr.nnz)
    pos = positions(csr, oracle.element_dofs(topo, kind))
    ga_o, gb_o = grad_coefficients(nodes, elems, kind, topo, pos, wK, wM)
    gn_o = grad_nodes(nodes, elems, kind, topo, pos, wK, wM, a, b)
    tn, te, ta, tb = dev_tensors(nodes, elems, a, b)
    mesh = fem.Mesh(tn, te)
    mesh.pattern(kind)
    tK = torch.tensor(wK, device=tn.device)
    tM = torch.tensor(wM, device=tn.device)
    gn, ga, gb = fem.assemble_backward(mesh, kind, tn, ta, tb, tK, tM)
    leaves = [t.clone().requires_grad_(True) for t in (tn, ta, tb)]
    K, M = fem.assemble(mesh, kind, *leaves)
    assert K.requires_grad
    ((tK * K).sum() + (tM * M).sum()).backward()
    mesh.status()
    assert torch.equal(leaves[0].grad, gn) and torch.equal(leaves[1].grad, ga) and torch.equal(leaves[2].grad, gb)
    for got, ref, nm in ((ga, ga_o, "a"), (gb, gb_o, "b"), (gn, gn_o, "x")):
        got = got.cpu().numpy()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        say(f"    dL/d{nm}: max rel err {err:.2e}")
        assert err <= GTOL, (nm, err)


@pytest.mark.parametrize("case", ["ned3", "rt3"])
def test_assemble_gradient_of_one_matrix(case):
    """A loss of K alone (M gets no gradient: it reaches the backward as None,
    a NULL weight array read as 0, with no zero tensor formed): the gradients
    equal fem_assemble_backward's with gM = NULL bitwise and the oracle's with
    gM = 0 within 1e-12."""
    import torch
    import paper_1409_4618_amd as fem
    nodes, elems, kind, a, b, rng = make_case(case, 23)
    say(f"[gpu] gradient of a loss of K only: {case}")
    csr, topo = oracle.assemble(nodes, elems, kind, a=a, b=b)
    wK = rng.normal(size=csr.nnz)
    zero = np.zeros(csr.nnz)
    pos = positions(csr, oracle.element_dofs(topo, kind))
    ga_o, gb_o = grad_coefficients(nodes, elems, kind, topo, pos, wK, zero)
    gn_o = grad_nodes(nodes, elems, kind, topo, pos, wK, zero, a, b)
    tn, te, ta, tb = dev_tensors(nodes, elems, a, b)
    mesh = fem.Mesh(tn, te)
    tK = torch.tensor(wK, device=tn.device)
    gn, ga, gb = fem.assemble_backward(mesh, kind, tn, ta, tb, tK, None)
    leaves = [t.clone().requires_grad_(True) for t in (tn, ta, tb)]
    K, M = fem.assemble(mesh, kind, *leaves)
    (tK * K).sum().backward()
    mesh.status()
    assert torch.equal(leaves[0].grad, gn) and torch.equal(leaves[1].grad, ga) and torch.equal(leaves[2].grad, gb)
    assert not gb.any()
    for got, ref, nm in ((ga, ga_o, "a"), (gn, gn_o, "x")):
        got = got.cpu().numpy()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        say(f"    dL/d{nm}: max rel err {err:.2e}")
        assert err <= GTOL, (nm, err)


@pytest.mark.parametrize("case", ["ned3", "rt3", "ned2"])
def test_csr_matvec(case):
    """fem_csr_matvec: alpha K x + beta M x and alpha K x against the oracle
    matrices' products (1e-12 relative), deterministic."""
    import torch
    import paper_1409_4618_amd as fem
    nodes, elems, kind, a, b, rng = make_case(case, 19)
    say(f"[gpu] CSR matvec: {case}")
    csr, _ = oracle.assemble(nodes, elems, kind, a=a, b=b)
    x = rng.normal(size=csr.n_rows)
    tn, te, ta, tb = dev_tensors(nodes, elems, a, b)
    mesh = fem.Mesh(tn, te)
    rowptr, colind = mesh.pattern(kind)
    K, M = fem.assemble(mesh, kind, tn, ta, tb)
    tx = torch.tensor(x, device=tn.device)
    y = fem.csr_matvec(rowptr, colind, K, tx, B=M, alpha=0.5, beta=-2.0)
    y2 = fem.csr_matvec(rowptr, colind, K, tx, B=M, alpha=0.5, beta=-2.0)
    assert torch.equal(y, y2)
    ref = 0.5 * (csr.scipy("K") @ x) - 2.0 * (csr.scipy("M") @ x)
    err = np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()
    yk = fem.csr_matvec(rowptr, colind, K, tx, alpha=1.5)
    refk = 1.5 * (csr.scipy("K") @ x)
    errk = np.abs(yk.cpu().numpy() - refk).max() / np.abs(refk).max()
    say(f"    rel err {err:.2e} (K and M), {errk:.2e} (K only)")
    assert err <= 1e-12 and errk <= 1e-12
