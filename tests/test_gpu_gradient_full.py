"""The adjoint at the full forward + backward size (Kuhn 96^3, 3D Nedelec,
5,308,416 tets; L = u^T (K(a) + M(b)) u, u ~ N(0, 1) per edge), in the launch
configuration bench.py times:

* the quadratic-form entry point equal, up to rounding (1e-12 of the largest
  value), to the general one with the materialised weights u_row u_col;
* sampled elements and vertices against the oracle: dL/da, dL/db of 256
  random elements and dL/dx of 64 random vertices, computed by the oracle on
  the sub-mesh of those elements and of every element around those vertices,
  with the weights u_I u_J of its own global numbering;
* identities that hold at any size, over the whole output: homogeneity in the
  coefficients (sum a dL/da = u^T K u, sum b dL/db = u^T M u), invariance of L
  under translations and rotations (sum_v dL/dx_v = 0, sum_v x_v x dL/dx_v = 0)
  and its scaling degree (sum_v x_v . dL/dx_v = -u^T K u + u^T M u, since K
  scales as 1/h and M as h).
"""
import dataclasses

import numpy as np
import pytest

import meshgen as mg
import oracle
from gpu_util import say
from oracle.gradient import grad_coefficients, grad_nodes

pytestmark = pytest.mark.gpu

GTOL = 1e-12


def test_full_size_adjoint():
    import torch
    import paper_1409_4618_amd as fem
    p = mg.kuhn96_ned_grad()
    say(f"[gpu] adjoint at full size: T={p.T} V={p.nodes.shape[0]}")
    d = torch.device("cuda:0")
    tn = torch.tensor(p.nodes, device=d)
    te = torch.tensor(p.elems, device=d)
    ta = torch.tensor(p.a, device=d)
    tb = torch.tensor(p.b, device=d)
    mesh = fem.Mesh(tn, te)
    rowptr, colind = mesh.pattern(p.kind)
    tu = torch.tensor(p.u, device=d)
    rows = torch.repeat_interleave(torch.arange(rowptr.numel() - 1, device=d), torch.diff(rowptr))
    w = tu[rows] * tu[colind.long()]
    del rows
    K, M = fem.assemble(mesh, p.kind, tn, ta, tb)
    gn, ga, gb = fem.assemble_backward(mesh, p.kind, tn, ta, tb, w, w)
    mesh.status()
    qn, qa, qb = fem.assemble_backward_quadratic(mesh, p.kind, tn, ta, tb, tu)
    mesh.status()
    for q, g, nm in ((qa, ga, "a"), (qb, gb, "b"), (qn, gn, "x")):
        err = float((q - g).abs().max()) / float(g.abs().max())
        say(f"    quadratic vs general dL/d{nm}: {err:.2e}")
        assert err <= 1e-12, (nm, err)
    del qn, qa, qb
    LK = float((w * K).sum())
    LM = float((w * M).sum())
    del K, M, w

    # identities over the whole output
    s1 = ta * ga
    s2 = tb * gb
    e1 = abs(float(s1.sum()) - LK) / float(s1.abs().sum())
    e2 = abs(float(s2.sum()) - LM) / float(s2.abs().sum())
    say(f"    sum a dL/da vs u^T K u: {e1:.2e}; sum b dL/db vs u^T M u: {e2:.2e}")
    assert e1 <= 1e-12 and e2 <= 1e-12
    gsum = gn.sum(dim=0)
    e3 = float(gsum.abs().max()) / float(gn.abs().sum())
    rot = torch.linalg.cross(tn, gn, dim=1)
    e4 = float(rot.sum(dim=0).abs().max()) / float(rot.abs().sum())
    xg = (tn * gn).sum(dim=1)
    e5 = abs(float(xg.sum()) - (-LK + LM)) / float(xg.abs().sum())
    say(f"    translation {e3:.2e}, rotation {e4:.2e}, scaling {e5:.2e}")
    assert e3 <= 1e-12 and e4 <= 1e-12 and e5 <= 1e-12

    # sampled elements and vertices against the oracle
    rng = np.random.default_rng(77)
    T, V = p.T, p.nodes.shape[0]
    topo = oracle.build_topology(p.elems, V)
    samp_e = rng.choice(T, size=256, replace=False)
    samp_v = rng.choice(V, size=64, replace=False)
    around = np.flatnonzero(np.isin(p.elems, samp_v).any(axis=1))
    sub = np.unique(np.concatenate([samp_e, around]))
    say(f"    oracle on a sub-mesh of {sub.size} elements")
    sub_topo = dataclasses.replace(topo, elems2edges=topo.elems2edges[sub], signs_e=topo.signs_e[sub],
                                   elems2faces=None if topo.elems2faces is None else topo.elems2faces[sub],
                                   signs_f=None if topo.signs_f is None else topo.signs_f[sub])
    dofs = oracle.element_dofs(sub_topo, p.kind)
    n = dofs.shape[1]
    wloc = (p.u[dofs][:, :, None] * p.u[dofs][:, None, :]).reshape(-1)   # u_I u_J per local entry
    pos = np.arange(sub.size * n * n).reshape(sub.size, n, n)
    ga_o, gb_o = grad_coefficients(p.nodes, p.elems[sub], p.kind, sub_topo, pos, wloc, wloc)
    gn_o = grad_nodes(p.nodes, p.elems[sub], p.kind, sub_topo, pos, wloc, wloc, p.a[sub], p.b[sub])
    idx = np.searchsorted(sub, samp_e)
    ga_g = ga.cpu().numpy()[samp_e]
    gb_g = gb.cpu().numpy()[samp_e]
    gn_g = gn.cpu().numpy()[samp_v]
    ea = np.abs(ga_g - ga_o[idx]).max() / np.abs(ga_o[idx]).max()
    eb = np.abs(gb_g - gb_o[idx]).max() / np.abs(gb_o[idx]).max()
    ex = np.abs(gn_g - gn_o[samp_v]).max() / np.abs(gn_o[samp_v]).max()
    say(f"    sampled dL/da {ea:.2e}, dL/db {eb:.2e}, dL/dx {ex:.2e}")
    assert ea <= GTOL and eb <= GTOL and ex <= GTOL
