"""Python binding of libfem: lowest-order edge-element assembly on MI355X.

Every step runs in the HIP kernels of ``libfem.so`` (C ABI in include/fem.h);
this module only marshals arguments. PyTorch provides device memory, the
current HIP stream and the autograd hook.

    import paper_1409_4618_amd as fem
    mesh = fem.Mesh(nodes, elems)              # topology on the GPU
    K, M = fem.assemble(mesh, "ned", nodes, a, b)   # differentiable in nodes, a, b
    rowptr, colind = mesh.pattern("ned")
    K, M, L = fem.assemble_quadratic(mesh, "ned", nodes, a, b, u)
    L.backward()                               # the quadratic adjoint
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

from ._lib import (FEM_FN_BUBBLE_F, FEM_FN_BUBBLE_GRAD_U, FEM_FN_BUBBLE_U, FEM_FN_EDDY_CURL_E, FEM_FN_EDDY_E,
                   FEM_FN_EDDY_F, FEM_FN_POLYNOMIAL, FEM_NEDELEC, FEM_RAVIART_THOMAS, FemError, check, hip, lib)

__all__ = ["Mesh", "Batch", "assemble", "assemble_backward", "assemble_backward_quadratic", "FemAssemble", "FemError",
           "kind_code", "NED", "RT", "quadratic_value", "quadratic_value_noalloc", "quadratic_value_adjoint",
           "quadratic_form", "assemble_quadratic", "csr_matvec",
           "norm_L2", "load_vector", "field_error", "cg_solve", "default_quad_m",
           "FEM_FN_POLYNOMIAL", "FEM_FN_EDDY_E", "FEM_FN_EDDY_CURL_E", "FEM_FN_EDDY_F", "FEM_FN_BUBBLE_U",
           "FEM_FN_BUBBLE_GRAD_U", "FEM_FN_BUBBLE_F", "p1_pattern", "p1_assemble", "p1_load", "p1_dirichlet",
           "p1_grad_error", "rt_majorant_rhs", "majorant_terms"]

NED = "ned"
RT = "rt"


def kind_code(kind) -> int:
    if kind in (NED, "nedelec", FEM_NEDELEC):
        return FEM_NEDELEC
    if kind in (RT, "raviart-thomas", FEM_RAVIART_THOMAS):
        return FEM_RAVIART_THOMAS
    raise ValueError(f"unknown kind {kind!r}")


def _torch():
    import torch
    return torch


def _stream_ptr():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _check_dev(t, dtype, name, shape=None):
    if t is None:
        return None
    if t.is_cuda and t.dtype == dtype and t.is_contiguous() and (shape is None or t.shape == shape):
        return t  # the common case, in one test
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _copy_from_device(ptr: int, n: int, dtype):
    """Copy a borrowed library buffer into a new torch tensor (same device)."""
    torch = _torch()
    out = torch.empty(n, dtype=dtype, device="cuda")
    if n:
        nbytes = n * out.element_size()
        check(0 if hip().hipMemcpyAsync(ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ptr),
                                        nbytes, 3, _stream_ptr()) == 0 else 7, "hipMemcpyAsync")
    return out


class Mesh:
    """Topology handle (fem_topology): global edge / face numbering and sign data."""

    def __init__(self, nodes, elems):
        torch = _torch()
        if elems.dim() != 2 or elems.shape[1] not in (3, 4):
            raise ValueError("elems must be [T, 3] or [T, 4]")
        self.dim = int(elems.shape[1]) - 1
        _check_dev(nodes, torch.float64, "nodes")
        _check_dev(elems, torch.int32, "elems")
        if nodes.dim() != 2 or nodes.shape[1] != self.dim:
            raise ValueError(f"nodes must be [V, {self.dim}]")
        self._h = ctypes.c_void_p(0)
        L = lib()
        check(L.fem_topology(_ptr(nodes), nodes.shape[0], self.dim, _ptr(elems), elems.shape[0],
                             _stream_ptr(), ctypes.byref(self._h)), "fem_topology")
        V = ctypes.c_int64()
        T = ctypes.c_int64()
        E = ctypes.c_int64()
        F = ctypes.c_int64()
        d = ctypes.c_int()
        check(L.fem_mesh_counts(self._h, ctypes.byref(V), ctypes.byref(T), ctypes.byref(E),
                                ctypes.byref(F), ctypes.byref(d)), "fem_mesh_counts")
        self.n_nodes, self.n_elems, self.n_edges, self.n_faces = V.value, T.value, E.value, F.value
        self._patterns = {}

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().fem_mesh_destroy(h)
                h.value = None
            except Exception:
                pass

    def topology(self, names=None):
        """Copies of the topology arrays as device tensors (dict): all of them, or
        those in ``names``."""
        torch = _torch()
        ptrs = [ctypes.c_void_p() for _ in range(6)]
        check(lib().fem_mesh_topology(self._h, *[ctypes.byref(p) for p in ptrs]), "fem_mesh_topology")
        ne = 6 if self.dim == 3 else 3
        layout = {"edges2nodes": (0, 2, self.n_edges, torch.int32), "elems2edges": (1, ne, self.n_elems, torch.int32),
                  "signs_e": (2, ne, self.n_elems, torch.int8)}
        if self.dim == 3:
            layout.update({"faces2nodes": (3, 3, self.n_faces, torch.int32),
                           "elems2faces": (4, 4, self.n_elems, torch.int32),
                           "signs_f": (5, 4, self.n_elems, torch.int8)})
        if names is not None:
            unknown = set(names) - set(layout)
            if unknown:
                raise ValueError(f"unknown topology arrays: {sorted(unknown)}")
            layout = {k: layout[k] for k in names}
        return {k: _copy_from_device(ptrs[i].value, w * n, dt).view(-1, w) for k, (i, w, n, dt) in layout.items()}

    def pattern_info(self, kind):
        """(n_rows, nnz) of the CSR pattern of ``kind`` (built on first use)."""
        kc = kind_code(kind)
        if kc not in self._patterns:
            n = ctypes.c_int64()
            nnz = ctypes.c_int64()
            rp = ctypes.c_void_p()
            ci = ctypes.c_void_p()
            check(lib().fem_pattern(self._h, kc, _stream_ptr(), ctypes.byref(n), ctypes.byref(nnz),
                                    ctypes.byref(rp), ctypes.byref(ci)), "fem_pattern")
            self._patterns[kc] = (n.value, nnz.value, rp.value, ci.value)
        return self._patterns[kc][:2]

    def pattern_device(self, kind):
        """(rowptr, colind) device tensors of ``kind``'s pattern (copies, cached on
        the mesh object)."""
        kc = kind_code(kind)
        cache = self.__dict__.setdefault("_pattern_dev", {})
        if kc not in cache:
            cache[kc] = self.pattern(kind)
        return cache[kc]

    def pattern(self, kind):
        """Copies of (rowptr int64 [n_rows+1], colind int32 [nnz]) as device tensors."""
        torch = _torch()
        self.pattern_info(kind)
        n, nnz, rp, ci = self._patterns[kind_code(kind)]
        return (_copy_from_device(rp, n + 1, torch.int64), _copy_from_device(ci, nnz, torch.int32))

    def status(self):
        """Synchronise and raise if an asynchronous kernel flagged an error."""
        check(lib().fem_status_query(self._h), "fem_status_query")


def _check_inputs(mesh: Mesh, nodes, a, b):
    torch = _torch()
    _check_dev(nodes, torch.float64, "nodes", (mesh.n_nodes, mesh.dim))
    _check_dev(a, torch.float64, "a", (mesh.n_elems,))
    _check_dev(b, torch.float64, "b", (mesh.n_elems,))


def assemble_into(mesh: Mesh, kind, nodes, a, b, K, M):
    """fem_assemble into caller-provided outputs (no allocation)."""
    torch = _torch()
    _, nnz = mesh.pattern_info(kind)
    _check_inputs(mesh, nodes, a, b)
    _check_dev(K, torch.float64, "K", (nnz,))
    _check_dev(M, torch.float64, "M", (nnz,))
    check(lib().fem_assemble(mesh.handle, kind_code(kind), _ptr(nodes), _ptr(a), _ptr(b), _ptr(K),
                             _ptr(M), _stream_ptr()), "fem_assemble")


def _assemble_values(mesh: Mesh, kind, nodes, a=None, b=None):
    torch = _torch()
    _, nnz = mesh.pattern_info(kind)
    _check_inputs(mesh, nodes, a, b)
    K = torch.empty(nnz, dtype=torch.float64, device=nodes.device)
    M = torch.empty(nnz, dtype=torch.float64, device=nodes.device)
    assemble_into(mesh, kind, nodes, a, b, K, M)
    return K, M


def _needs_grad(*ts):
    torch = _torch()
    return torch.is_grad_enabled() and any(t is not None and t.requires_grad for t in ts)


def assemble(mesh: Mesh, kind, nodes, a=None, b=None):
    """Values (K, M) of K(a), M(b) on ``mesh.pattern(kind)``: f64 device tensors [nnz].

    Differentiable: when nodes, a or b require grad, the values come from the
    autograd Function FemAssemble, whose backward is fem_assemble_backward."""
    if _needs_grad(nodes, a, b):
        return FemAssemble().apply(nodes, a, b, mesh, kind)
    return _assemble_values(mesh, kind, nodes, a, b)


def quadratic_value(mesh: Mesh, kind, nodes, a, b, u):
    """L = u^T (K(a) + M(b)) u as a 0-dim device tensor (fem_quadratic_value; no
    gradient)."""
    torch = _torch()
    n_rows, _ = mesh.pattern_info(kind)
    _check_inputs(mesh, nodes, a, b)
    _check_dev(u, torch.float64, "u", (n_rows,))
    L = torch.empty((), dtype=torch.float64, device=nodes.device)
    check(lib().fem_quadratic_value(mesh.handle, kind_code(kind), _ptr(nodes), _ptr(a), _ptr(b), _ptr(u),
                                    _ptr(L), _stream_ptr()), "fem_quadratic_value")
    return L


def quadratic_value_noalloc(mesh: Mesh, kind, nodes, a, b, u, out):
    """L = u^T (K(a) + M(b)) u into the caller's 0-dim device tensor ``out``
    (fem_quadratic_value_noalloc: no device allocation by the library or here;
    meshes of at most 2^27 elements; calls overlapping on one GPU race)."""
    torch = _torch()
    n_rows, _ = mesh.pattern_info(kind)
    _check_inputs(mesh, nodes, a, b)
    _check_dev(u, torch.float64, "u", (n_rows,))
    _check_dev(out, torch.float64, "out", ())
    check(lib().fem_quadratic_value_noalloc(mesh.handle, kind_code(kind), _ptr(nodes), _ptr(a), _ptr(b),
                                            _ptr(u), _ptr(out), _stream_ptr()), "fem_quadratic_value_noalloc")
    return out


def csr_matvec(rowptr, colind, A, x, B=None, alpha=1.0, beta=1.0, out=None):
    """y = alpha A x + beta B x on a CSR pattern (fem_csr_matvec)."""
    torch = _torch()
    n = rowptr.numel() - 1
    nnz = colind.numel()
    _check_dev(rowptr, torch.int64, "rowptr")
    _check_dev(colind, torch.int32, "colind")
    _check_dev(A, torch.float64, "A", (nnz,))
    _check_dev(B, torch.float64, "B", (nnz,))
    _check_dev(x, torch.float64, "x")
    y = torch.empty(n, dtype=torch.float64, device=A.device) if out is None else out
    _check_dev(y, torch.float64, "y", (n,))
    check(lib().fem_csr_matvec(n, _ptr(rowptr), _ptr(colind), _ptr(A), _ptr(B), float(alpha), float(beta),
                               _ptr(x), _ptr(y), _stream_ptr()), "fem_csr_matvec")
    return y


def default_quad_m(dim: int) -> int:
    """Gauss-Legendre points per direction of the conical rule whose degree
    reaches 6, the order of the paper's norm_L2 (2D: 4 -> degree 6; 3D: 5 -> 7)."""
    return 4 if dim == 2 else 5


def _fn_params(params):
    """Host array of polynomial parameters (flat sequence of floats) -> (ptr, n)."""
    if params is None:
        return None, 0
    flat = [float(v) for v in params]
    arr = (ctypes.c_double * len(flat))(*flat)
    return arr, len(flat)


def norm_L2(mesh: Mesh, nodes, fn, params=None, quad_m=None, per_elem=False):
    """(per-element ||f||_K^2 [T] or None, total ||f||^2 0-dim tensor) of a
    catalogue function (fem_norm_L2, Section 3.1)."""
    torch = _torch()
    _check_dev(nodes, torch.float64, "nodes", (mesh.n_nodes, mesh.dim))
    arr, n = _fn_params(params)
    per = torch.empty(mesh.n_elems, dtype=torch.float64, device=nodes.device) if per_elem else None
    tot = torch.empty((), dtype=torch.float64, device=nodes.device)
    check(lib().fem_norm_L2(mesh.handle, _ptr(nodes), int(fn), arr, n,
                            default_quad_m(mesh.dim) if quad_m is None else int(quad_m), _ptr(per), _ptr(tot),
                            _stream_ptr()), "fem_norm_L2")
    return per, tot


def load_vector(mesh: Mesh, kind, nodes, fn, params=None, quad_m=None):
    """f_i = int F . eta_i over the Nedelec basis (fem_load_vector) -> [n_edges]."""
    torch = _torch()
    _check_dev(nodes, torch.float64, "nodes", (mesh.n_nodes, mesh.dim))
    arr, n = _fn_params(params)
    f = torch.empty(mesh.n_edges, dtype=torch.float64, device=nodes.device)
    check(lib().fem_load_vector(mesh.handle, kind_code(kind), _ptr(nodes), int(fn), arr, n,
                                default_quad_m(mesh.dim) if quad_m is None else int(quad_m), _ptr(f),
                                _stream_ptr()), "fem_load_vector")
    return f


def field_error(mesh: Mesh, kind, nodes, v, field, curl, params=None, quad_m=None, per_elem=False):
    """(per-element [T] or None, total 0-dim tensor) of
    int |E - v_h|^2 + |curl E - curl v_h|^2 (fem_field_error)."""
    torch = _torch()
    _check_dev(nodes, torch.float64, "nodes", (mesh.n_nodes, mesh.dim))
    _check_dev(v, torch.float64, "v", (mesh.n_edges,))
    arr, n = _fn_params(params)
    per = torch.empty(mesh.n_elems, dtype=torch.float64, device=nodes.device) if per_elem else None
    tot = torch.empty((), dtype=torch.float64, device=nodes.device)
    check(lib().fem_field_error(mesh.handle, kind_code(kind), _ptr(nodes), _ptr(v), int(field), int(curl), arr, n,
                                default_quad_m(mesh.dim) if quad_m is None else int(quad_m), _ptr(per), _ptr(tot),
                                _stream_ptr()), "fem_field_error")
    return per, tot


def cg_solve(rowptr, colind, A, rhs, B=None, ca=1.0, cb=1.0, x0=None, rtol=1e-12, max_iter=None):
    """Solve (ca A + cb B) x = rhs by Jacobi-preconditioned CG (fem_cg_solve).
    Returns (x, iterations, true relative residual)."""
    torch = _torch()
    n = rowptr.numel() - 1
    nnz = colind.numel()
    _check_dev(rowptr, torch.int64, "rowptr")
    _check_dev(colind, torch.int32, "colind")
    _check_dev(A, torch.float64, "A", (nnz,))
    _check_dev(B, torch.float64, "B", (nnz,))
    _check_dev(rhs, torch.float64, "rhs", (n,))
    x = torch.zeros(n, dtype=torch.float64, device=A.device) if x0 is None else x0.clone()
    _check_dev(x, torch.float64, "x", (n,))
    it = ctypes.c_int64()
    res = ctypes.c_double()
    check(lib().fem_cg_solve(n, _ptr(rowptr), _ptr(colind), _ptr(A), _ptr(B), float(ca), float(cb), _ptr(rhs),
                             _ptr(x), float(rtol), int(10 * n if max_iter is None else max_iter), _stream_ptr(),
                             ctypes.byref(it), ctypes.byref(res)), "fem_cg_solve")
    return x, it.value, res.value


def p1_pattern(mesh: Mesh):
    """(rowptr, colind) copies of the nodal P1 pattern (fem_p1_pattern)."""
    torch = _torch()
    cache = mesh.__dict__.setdefault("_p1", None)
    if cache is None:
        n = ctypes.c_int64()
        nnz = ctypes.c_int64()
        rp = ctypes.c_void_p()
        ci = ctypes.c_void_p()
        check(lib().fem_p1_pattern(mesh.handle, _stream_ptr(), ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(rp),
                                   ctypes.byref(ci)), "fem_p1_pattern")
        cache = (_copy_from_device(rp.value, n.value + 1, torch.int64), _copy_from_device(ci.value, nnz.value,
                                                                                          torch.int32))
        mesh.__dict__["_p1"] = cache
    return cache


def p1_assemble(mesh: Mesh, nodes, a=None):
    """P1 stiffness values [nnz] on p1_pattern(mesh) (fem_p1_assemble)."""
    torch = _torch()
    rowptr, colind = p1_pattern(mesh)
    _check_dev(nodes, torch.float64, "nodes", (mesh.n_nodes, mesh.dim))
    _check_dev(a, torch.float64, "a", (mesh.n_elems,))
    K = torch.empty(colind.numel(), dtype=torch.float64, device=nodes.device)
    check(lib().fem_p1_assemble(mesh.handle, _ptr(nodes), _ptr(a), _ptr(K), _stream_ptr()), "fem_p1_assemble")
    return K


def p1_load(mesh: Mesh, nodes, fn, params=None, quad_m=None):
    """F_i = int f lambda_i [n_nodes] (fem_p1_load)."""
    torch = _torch()
    p1_pattern(mesh)
    _check_dev(nodes, torch.float64, "nodes", (mesh.n_nodes, mesh.dim))
    arr, n = _fn_params(params)
    F = torch.empty(mesh.n_nodes, dtype=torch.float64, device=nodes.device)
    check(lib().fem_p1_load(mesh.handle, _ptr(nodes), int(fn), arr, n,
                            default_quad_m(mesh.dim) if quad_m is None else int(quad_m), _ptr(F), _stream_ptr()),
          "fem_p1_load")
    return F


def p1_dirichlet(mesh: Mesh, K=None, rhs=None):
    """Eliminate the boundary nodes in place (fem_p1_dirichlet)."""
    torch = _torch()
    _, colind = p1_pattern(mesh)
    _check_dev(K, torch.float64, "K", (colind.numel(),))
    _check_dev(rhs, torch.float64, "rhs", (mesh.n_nodes,))
    check(lib().fem_p1_dirichlet(mesh.handle, _ptr(K), _ptr(rhs), _stream_ptr()), "fem_p1_dirichlet")


def p1_grad_error(mesh: Mesh, nodes, v, fn, params=None, quad_m=None, per_elem=False):
    """(per-element [T] or None, total 0-dim tensor) of int |g - grad v|^2 (fem_p1_grad_error)."""
    torch = _torch()
    _check_dev(nodes, torch.float64, "nodes", (mesh.n_nodes, mesh.dim))
    _check_dev(v, torch.float64, "v", (mesh.n_nodes,))
    arr, n = _fn_params(params)
    per = torch.empty(mesh.n_elems, dtype=torch.float64, device=nodes.device) if per_elem else None
    tot = torch.empty((), dtype=torch.float64, device=nodes.device)
    check(lib().fem_p1_grad_error(mesh.handle, _ptr(nodes), _ptr(v), int(fn), arr, n,
                                  default_quad_m(mesh.dim) if quad_m is None else int(quad_m), _ptr(per), _ptr(tot),
                                  _stream_ptr()), "fem_p1_grad_error")
    return per, tot


def rt_majorant_rhs(mesh: Mesh, nodes, v, fn, c_div, c_grad, params=None, quad_m=None, out=None):
    """c_div int f div phi_i + c_grad int grad v . phi_i over the RT basis (fem_rt_majorant_rhs)."""
    torch = _torch()
    n_rows, _ = mesh.pattern_info(RT)
    _check_dev(nodes, torch.float64, "nodes", (mesh.n_nodes, mesh.dim))
    _check_dev(v, torch.float64, "v", (mesh.n_nodes,))
    arr, n = _fn_params(params)
    rhs = torch.empty(n_rows, dtype=torch.float64, device=nodes.device) if out is None else out
    _check_dev(rhs, torch.float64, "rhs", (n_rows,))
    check(lib().fem_rt_majorant_rhs(mesh.handle, _ptr(nodes), _ptr(v), int(fn), arr, n,
                                    default_quad_m(mesh.dim) if quad_m is None else int(quad_m), float(c_div),
                                    float(c_grad), _ptr(rhs), _stream_ptr()), "fem_rt_majorant_rhs")
    return rhs


def majorant_terms(mesh: Mesh, nodes, v, y, fn, params=None, quad_m=None):
    """Device tensor [2]: ||grad v - y||^2 and ||div y + f||^2 (fem_majorant_terms)."""
    torch = _torch()
    n_rows, _ = mesh.pattern_info(RT)
    _check_dev(nodes, torch.float64, "nodes", (mesh.n_nodes, mesh.dim))
    _check_dev(v, torch.float64, "v", (mesh.n_nodes,))
    _check_dev(y, torch.float64, "y", (n_rows,))
    arr, n = _fn_params(params)
    out = torch.empty(2, dtype=torch.float64, device=nodes.device)
    check(lib().fem_majorant_terms(mesh.handle, _ptr(nodes), _ptr(v), _ptr(y), int(fn), arr, n,
                                   default_quad_m(mesh.dim) if quad_m is None else int(quad_m), _ptr(out),
                                   _stream_ptr()), "fem_majorant_terms")
    return out


def assemble_backward(mesh: Mesh, kind, nodes, a, b, gK, gM, need_a=True, need_b=True,
                      need_nodes=True):
    """Adjoint: (dL/dnodes, dL/da, dL/db) for L = gK . K(a) + gM . M(b)."""
    torch = _torch()
    _, nnz = mesh.pattern_info(kind)
    _check_inputs(mesh, nodes, a, b)
    _check_dev(gK, torch.float64, "gK", (nnz,))
    _check_dev(gM, torch.float64, "gM", (nnz,))
    dev = nodes.device
    ga = torch.empty(mesh.n_elems, dtype=torch.float64, device=dev) if need_a else None
    gb = torch.empty(mesh.n_elems, dtype=torch.float64, device=dev) if need_b else None
    gn = torch.empty_like(nodes) if need_nodes else None
    check(lib().fem_assemble_backward(mesh.handle, kind_code(kind), _ptr(nodes), _ptr(a), _ptr(b),
                                      _ptr(gK), _ptr(gM), _ptr(ga), _ptr(gb), _ptr(gn),
                                      _stream_ptr()), "fem_assemble_backward")
    return gn, ga, gb


def assemble_backward_quadratic(mesh: Mesh, kind, nodes, a, b, u, need_a=True, need_b=True,
                                need_nodes=True):
    """Adjoint of L = u^T (K(a) + M(b)) u: (dL/dnodes, dL/da, dL/db), the same as
    assemble_backward with gK = gM = u_row u_col, without materialising them."""
    torch = _torch()
    n_rows, _ = mesh.pattern_info(kind)
    _check_inputs(mesh, nodes, a, b)
    _check_dev(u, torch.float64, "u", (n_rows,))
    dev = nodes.device
    ga = torch.empty(mesh.n_elems, dtype=torch.float64, device=dev) if need_a else None
    gb = torch.empty(mesh.n_elems, dtype=torch.float64, device=dev) if need_b else None
    gn = torch.empty_like(nodes) if need_nodes else None
    check(lib().fem_assemble_backward_quadratic(mesh.handle, kind_code(kind), _ptr(nodes), _ptr(a), _ptr(b),
                                                _ptr(u), _ptr(ga), _ptr(gb), _ptr(gn), _stream_ptr()),
          "fem_assemble_backward_quadratic")
    return gn, ga, gb


def quadratic_value_adjoint(mesh: Mesh, kind, nodes, a, b, u, need_a=True, need_b=True, need_nodes=True):
    """(L, dL/dnodes, dL/da, dL/db) of L = u^T (K(a) + M(b)) u from one pass
    (fem_quadratic_value_adjoint): the forward value with its adjoint ready for
    a backward pass."""
    torch = _torch()
    n_rows, _ = mesh.pattern_info(kind)
    _check_inputs(mesh, nodes, a, b)
    _check_dev(u, torch.float64, "u", (n_rows,))
    dev = nodes.device
    L = torch.empty((), dtype=torch.float64, device=dev)
    ga = torch.empty(mesh.n_elems, dtype=torch.float64, device=dev) if need_a else None
    gb = torch.empty(mesh.n_elems, dtype=torch.float64, device=dev) if need_b else None
    gn = torch.empty_like(nodes) if need_nodes else None
    check(lib().fem_quadratic_value_adjoint(mesh.handle, kind_code(kind), _ptr(nodes), _ptr(a), _ptr(b), _ptr(u),
                                            _ptr(L), _ptr(ga), _ptr(gb), _ptr(gn), _stream_ptr()),
          "fem_quadratic_value_adjoint")
    return L, gn, ga, gb


def _autograd_function():
    torch = _torch()

    class FemAssemble(torch.autograd.Function):
        """(nodes, a, b) -> (K values, M values) with the hand-written adjoint."""

        @staticmethod
        def forward(ctx, nodes, a, b, mesh, kind):
            K, M = _assemble_values(mesh, kind, nodes, a, b)
            ctx.mesh = mesh
            ctx.kind = kind
            ctx.save_for_backward(nodes, a, b)
            # an output without a gradient reaches backward as None (a NULL
            # weight array to the adjoint, which reads it as 0) instead of an
            # nnz-sized zero tensor
            ctx.set_materialize_grads(False)
            return K, M

        @staticmethod
        def backward(ctx, gK, gM):
            nodes, a, b = ctx.saved_tensors
            if gK is None and gM is None:
                return None, None, None, None, None
            gK = None if gK is None else gK.contiguous()
            gM = None if gM is None else gM.contiguous()
            gn, ga, gb = assemble_backward(ctx.mesh, ctx.kind, nodes, a, b, gK, gM,
                                           need_a=ctx.needs_input_grad[1],
                                           need_b=ctx.needs_input_grad[2],
                                           need_nodes=ctx.needs_input_grad[0])
            return gn, ga, gb, None, None

    return FemAssemble


def _quadratic_forward(ctx, nodes, a, b, u, mesh, kind):
    """L, and when nodes, a or b need a gradient, their derivatives from the
    same pass (fem_quadratic_value_adjoint), kept for the backward."""
    need_x, need_a, need_b = ctx.needs_input_grad[:3]
    ctx.adj = None
    if need_x or need_a or need_b:
        L, gn, ga, gb = quadratic_value_adjoint(mesh, kind, nodes, a, b, u, need_a=need_a, need_b=need_b,
                                                need_nodes=need_x)
        ctx.adj = (gn, ga, gb)
    else:
        L = quadratic_value(mesh, kind, nodes, a, b, u)
    return L


def _quadratic_backward(ctx, gL):
    """Gradients of L = u^T (K(a) + M(b)) u, scaled by the upstream gL: the
    quadratic adjoint for nodes, a and b (computed by the forward pass), and
    2 (K + M) u for u (K and M from the forward when it kept them, else
    assembled here)."""
    nodes, a, b, u = ctx.saved_tensors[:4]
    mesh, kind = ctx.mesh, ctx.kind
    need_u = ctx.needs_input_grad[3]
    gn = ga = gb = gu = None
    if ctx.adj is not None:
        # out of place (a graph kept with retain_graph=True may be differentiated
        # again), all three in one multi-tensor launch
        have = [g for g in ctx.adj if g is not None]
        scaled = iter(_torch()._foreach_mul(have, gL)) if have else iter(())
        gn, ga, gb = (None if g is None else next(scaled) for g in ctx.adj)
    if need_u:
        if len(ctx.saved_tensors) > 4:
            K, M = ctx.saved_tensors[4:6]
        else:
            K, M = _assemble_values(mesh, kind, nodes, a, b)
        rowptr, colind = mesh.pattern_device(kind)
        gu = csr_matvec(rowptr, colind, K, u, B=M, alpha=2.0, beta=2.0)
    # chain rule: the adjoint kernels compute dL/d(.); the upstream factor
    # (1 for L.backward()) multiplies them
    if gu is not None:
        gu.mul_(gL)
    return gn, ga, gb, gu


def _quadratic_functions():
    torch = _torch()

    class FemQuadratic(torch.autograd.Function):
        """(nodes, a, b, u) -> L = u^T (K(a) + M(b)) u (fem_quadratic_value),
        backward by the quadratic adjoint (fem_assemble_backward_quadratic)."""

        @staticmethod
        def forward(ctx, nodes, a, b, u, mesh, kind):
            L = _quadratic_forward(ctx, nodes, a, b, u, mesh, kind)
            ctx.mesh = mesh
            ctx.kind = kind
            ctx.save_for_backward(nodes, a, b, u)
            return L

        @staticmethod
        def backward(ctx, gL):
            return (*_quadratic_backward(ctx, gL), None, None)

    class FemAssembleQuadratic(torch.autograd.Function):
        """(nodes, a, b, u) -> (K values, M values, L): the assembled matrices
        (fem_assemble; returned for the caller, not differentiated) and the
        differentiable quadratic form L = u^T (K(a) + M(b)) u."""

        @staticmethod
        def forward(ctx, nodes, a, b, u, mesh, kind):
            K, M = _assemble_values(mesh, kind, nodes, a, b)
            L = _quadratic_forward(ctx, nodes, a, b, u, mesh, kind)
            ctx.mesh = mesh
            ctx.kind = kind
            ctx.mark_non_differentiable(K, M)
            # K and M get no gradient: without this, autograd would fill two
            # nnz-sized zero tensors for them on every backward
            ctx.set_materialize_grads(False)
            if ctx.needs_input_grad[3]:
                ctx.save_for_backward(nodes, a, b, u, K, M)
            else:
                ctx.save_for_backward(nodes, a, b, u)
            return K, M, L

        @staticmethod
        def backward(ctx, gK, gM, gL):
            if gL is None:
                return (None,) * 6
            return (*_quadratic_backward(ctx, gL), None, None)

    return FemQuadratic, FemAssembleQuadratic


_FA = None
_FQ = None


def FemAssemble():
    global _FA
    if _FA is None:
        _FA = _autograd_function()
    return _FA


def _fq():
    global _FQ
    if _FQ is None:
        _FQ = _quadratic_functions()
    return _FQ


def assemble_autograd(mesh: Mesh, kind, nodes, a, b):
    """Differentiable (K, M) values with respect to nodes, a and b."""
    return FemAssemble().apply(nodes, a, b, mesh, kind)


def quadratic_form(mesh: Mesh, kind, nodes, a, b, u):
    """Differentiable L = u^T (K(a) + M(b)) u (0-dim tensor) with respect to
    nodes, a, b and u, without assembling K and M in the forward."""
    return _fq()[0].apply(nodes, a, b, u, mesh, kind)


def assemble_quadratic(mesh: Mesh, kind, nodes, a, b, u):
    """(K, M, L): the assembled values of K(a), M(b) and the differentiable
    L = u^T (K(a) + M(b)) u, whose backward is the quadratic adjoint."""
    return _fq()[1].apply(nodes, a, b, u, mesh, kind)


class Batch:
    """Many meshes in one persistent launch (fem_batch_*)."""

    def __init__(self, meshes: Sequence[Mesh], kinds: Sequence):
        self.meshes = list(meshes)
        self.kinds = [kind_code(k) for k in kinds]
        for m, k in zip(self.meshes, self.kinds):
            m.pattern_info(k)
        n = len(self.meshes)
        handles = (ctypes.c_void_p * n)(*[m.handle.value for m in self.meshes])
        kinds_arr = (ctypes.c_int * n)(*self.kinds)
        self._h = ctypes.c_void_p(0)
        check(lib().fem_batch_create(handles, kinds_arr, n, ctypes.byref(self._h)), "fem_batch_create")
        self._keep = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().fem_batch_destroy(h)
                h.value = None
            except Exception:
                pass

    def bind(self, nodes, a, b, K, M):
        """Per-mesh device tensors (sequences of length n; a, b, K, M entries may be None)."""
        torch = _torch()
        n = len(self.meshes)
        nodes, a, b, K, M = (list(x) for x in (nodes, a, b, K, M))
        if any(len(x) != n for x in (nodes, a, b, K, M)):
            raise ValueError(f"bind needs {n} entries per argument")
        for i, (m, k) in enumerate(zip(self.meshes, self.kinds)):
            _, nnz = m.pattern_info(k)
            if nodes[i] is None:
                raise ValueError(f"nodes[{i}] is None")
            _check_inputs(m, nodes[i], a[i], b[i])
            _check_dev(K[i], torch.float64, f"K[{i}]", (nnz,))
            _check_dev(M[i], torch.float64, f"M[{i}]", (nnz,))

        def arr(ts):
            return (ctypes.c_void_p * n)(*[(0 if t is None else t.data_ptr()) for t in ts])

        self._keep = (nodes, a, b, K, M)
        check(lib().fem_batch_bind(self._h, arr(nodes), arr(a), arr(b), arr(K), arr(M)), "fem_batch_bind")

    def tune(self, cache_path: Optional[str] = None):
        p = None if cache_path is None else cache_path.encode()
        check(lib().fem_batch_tune(self._h, p, _stream_ptr()), "fem_batch_tune")

    def set_config(self, rows_per_tile: int, schedule: int, threads: int = 256):
        """Tiling (0 = element-major, or 64/128/256 rows), schedule (0..2; with
        element-major tiles also 3..4, one launch per element kind) and, for
        element-major tiles, the workgroup size (128 or 256)."""
        check(lib().fem_batch_set_config(self._h, rows_per_tile, schedule, threads), "fem_batch_set_config")

    def config(self):
        R = ctypes.c_int()
        s = ctypes.c_int()
        t = ctypes.c_int()
        nw = ctypes.c_int64()
        g = ctypes.c_int()
        check(lib().fem_batch_config(self._h, ctypes.byref(R), ctypes.byref(s), ctypes.byref(t), ctypes.byref(nw),
                                     ctypes.byref(g)), "fem_batch_config")
        return {"rows_per_tile": R.value, "schedule": s.value, "threads": t.value, "n_work": nw.value,
                "grid": g.value}

    def assemble(self):
        check(lib().fem_batch_assemble(self._h, _stream_ptr()), "fem_batch_assemble")

    def graph_launch(self):
        check(lib().fem_batch_graph_launch(self._h, _stream_ptr()), "fem_batch_graph_launch")
