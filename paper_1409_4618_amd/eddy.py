"""The 2D eddy-current example of Section 4.2 on the GPU.

curl_vec(mu^-1 curl E) + kappa E = F in the unit square with mu = kappa = 1 and
the natural boundary condition on the whole boundary, discretised with 2D
lowest-order Nedelec elements: (K(1/mu) + M(kappa)) v = f. Every step runs in
libfem's kernels: the assembly (fem_assemble), the load vector
f_i = int F . eta_i (fem_load_vector), the Jacobi-preconditioned conjugate
gradients (fem_cg_solve) and the energy error
sqrt(||E - v||^2 + ||curl(E - v)||^2) against the example's exact solution
(fem_field_error), the quantity of the paper's eddy table.
"""
from __future__ import annotations

import math

from . import (FEM_FN_EDDY_CURL_E, FEM_FN_EDDY_E, FEM_FN_EDDY_F, Mesh, _assemble_values, cg_solve, field_error,
               load_vector)


def eddy_current(mesh: Mesh, nodes, quad_m: int = 4, rtol: float = 1e-12, max_iter=None):
    """Solve the example on ``mesh`` (a 2D triangle mesh of the unit square
    whose edges follow the diagonal x1 = x2, so that every element lies on one
    side of the jump of E). Returns a dict with K, M, the load vector f, the
    edge values v, the CG iteration count and residual, and the energy error."""
    if mesh.dim != 2:
        raise ValueError("the eddy-current example is two-dimensional")
    K, M = _assemble_values(mesh, "ned", nodes)
    rowptr, colind = mesh.pattern_device("ned")
    f = load_vector(mesh, "ned", nodes, FEM_FN_EDDY_F, quad_m=quad_m)
    v, iters, res = cg_solve(rowptr, colind, K, f, B=M, rtol=rtol, max_iter=max_iter)
    _, err2 = field_error(mesh, "ned", nodes, v, FEM_FN_EDDY_E, FEM_FN_EDDY_CURL_E, quad_m=quad_m)
    mesh.status()
    return dict(K=K, M=M, f=f, v=v, iters=iters, rel_resid=res, error2=err2, error=math.sqrt(err2.item()))
