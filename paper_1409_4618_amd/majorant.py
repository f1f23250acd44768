"""Minimisation of the functional majorant (Section 4.1) on the GPU.

For -Lap u = f in the unit square / cube with u = 0 on the boundary (the
example's bubble u = prod_i x_i (x_i - 1)):
  1. v from linear nodal elements: fem_p1_assemble, fem_p1_load,
     fem_p1_dirichlet, then conjugate gradients (fem_cg_solve);
  2. for the current beta, y from the Raviart-Thomas discretisation of the
     quadratic problem of Section 4.1:
        ((1 + beta) C^2 K + (1 + 1/beta) M) y
            = -(1 + beta) C^2 int f div phi + (1 + 1/beta) int grad v . phi,
     K, M from fem_assemble, the right-hand side from fem_rt_majorant_rhs, CG;
  3. the terms ||grad v - y||^2, ||div y + f||^2 (fem_majorant_terms), the
     majorant M = sqrt((1 + 1/beta) a + (1 + beta) C^2 b) and the new
     beta = sqrt(a) / (C sqrt(b)) (Algorithm 1), until M changes by less than
     1e-4 relative to its previous value.
C = 1 / (pi sqrt(d)), the Friedrichs constant of the unit square / cube.
Every step runs in libfem's kernels; this module passes scalars between them.
"""
from __future__ import annotations

import math

from . import (FEM_FN_BUBBLE_F, FEM_FN_BUBBLE_GRAD_U, RT, Mesh, _assemble_values, cg_solve, majorant_terms,
               p1_assemble, p1_dirichlet, p1_grad_error, p1_load, p1_pattern, rt_majorant_rhs)


def friedrichs_constant(dim: int) -> float:
    return 1.0 / (math.pi * math.sqrt(dim))


def minimise(mesh: Mesh, nodes, beta0: float = 1.0, tol: float = 1e-4, max_iter: int = 20, rtol: float = 1e-12,
             quad_m=None):
    """Algorithm 1 of Section 4.1 on ``mesh``. Returns a dict with the P1 field v,
    its error ||grad(u - v)||, the CG iteration counts, and per iteration beta,
    the majorant, the efficiency index and y."""
    dim = mesh.dim
    C = friedrichs_constant(dim)
    rowptr_p1, colind_p1 = p1_pattern(mesh)
    Kp = p1_assemble(mesh, nodes)
    Fp = p1_load(mesh, nodes, FEM_FN_BUBBLE_F, quad_m=quad_m)
    p1_dirichlet(mesh, Kp, Fp)
    v, it_v, _ = cg_solve(rowptr_p1, colind_p1, Kp, Fp, rtol=rtol)
    _, e2 = p1_grad_error(mesh, nodes, v, FEM_FN_BUBBLE_GRAD_U, quad_m=quad_m)
    err = math.sqrt(e2.item())
    K, M = _assemble_values(mesh, RT, nodes)
    rowptr, colind = mesh.pattern_device(RT)
    beta = beta0
    prev = None
    iters = []
    y = None
    for _ in range(max_iter):
        cK = (1.0 + beta) * C * C
        cM = 1.0 + 1.0 / beta
        rhs = rt_majorant_rhs(mesh, nodes, v, FEM_FN_BUBBLE_F, -cK, cM, quad_m=quad_m)
        y, it_y, _ = cg_solve(rowptr, colind, K, rhs, B=M, ca=cK, cb=cM, x0=y, rtol=rtol)
        a2, b2 = (float(t) for t in majorant_terms(mesh, nodes, v, y, FEM_FN_BUBBLE_F, quad_m=quad_m).tolist())
        Mval = math.sqrt(cM * a2 + cK * b2)
        iters.append(dict(beta=beta, majorant=Mval, ieff=Mval / err, y=y, terms=(a2, b2), cg_iterations=it_y))
        if prev is not None and abs(prev - Mval) / prev < tol:
            break
        prev = Mval
        beta = math.sqrt(a2) / (C * math.sqrt(b2))
    mesh.status()
    return dict(v=v, error=err, cg_iterations_v=it_v, iterations=iters)
