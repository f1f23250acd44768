"""ctypes declarations of libfem's C ABI (include/fem.h).

Loading fails loudly if ``libfem.so`` has not been built: there is no fallback
implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# FEM_CHECK=1 selects the checked build (bounds checks in every kernel; same
# results, slower); the default is the production library.
LIB_PATH = os.path.join(HERE, "libfem_check.so" if os.environ.get("FEM_CHECK") == "1" else "libfem.so")

c_int64_p = ctypes.POINTER(ctypes.c_int64)
c_void_pp = ctypes.POINTER(ctypes.c_void_p)

FEM_NEDELEC = 0
FEM_RAVIART_THOMAS = 1

# fem_function
FEM_FN_POLYNOMIAL = 0
FEM_FN_EDDY_E = 1
FEM_FN_EDDY_CURL_E = 2
FEM_FN_EDDY_F = 3
FEM_FN_BUBBLE_U = 4
FEM_FN_BUBBLE_GRAD_U = 5
FEM_FN_BUBBLE_F = 6

STATUS_NAMES = {0: "FEM_OK", 1: "FEM_EINVAL", 2: "FEM_ERANGE", 3: "FEM_EDEGENERATE",
                4: "FEM_ENONFINITE", 5: "FEM_EOVERFLOW", 6: "FEM_ENOMEM", 7: "FEM_EHIP",
                8: "FEM_ENOTREADY"}

# (name, restype, argtypes) for every entry point declared in include/fem.h
SIGNATURES = [
    ("fem_topology", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                    ctypes.c_int64, ctypes.c_void_p, c_void_pp]),
    ("fem_mesh_counts", ctypes.c_int, [ctypes.c_void_p, c_int64_p, c_int64_p, c_int64_p, c_int64_p,
                                       ctypes.POINTER(ctypes.c_int)]),
    ("fem_mesh_topology", ctypes.c_int, [ctypes.c_void_p] + [c_void_pp] * 6),
    ("fem_pattern", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, c_int64_p, c_int64_p,
                                   c_void_pp, c_void_pp]),
    ("fem_assemble", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int] + [ctypes.c_void_p] * 6),
    ("fem_assemble_backward", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int] + [ctypes.c_void_p] * 9),
    ("fem_assemble_backward_quadratic", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int] + [ctypes.c_void_p] * 8),
    ("fem_quadratic_value", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int] + [ctypes.c_void_p] * 6),
    ("fem_quadratic_value_noalloc", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int] + [ctypes.c_void_p] * 6),
    ("fem_quadratic_value_adjoint", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int] + [ctypes.c_void_p] * 9),
    ("fem_csr_matvec", ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    ("fem_norm_L2", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("fem_load_vector", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    ("fem_field_error", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    ("fem_cg_solve", ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_double, ctypes.c_int64, ctypes.c_void_p, c_int64_p,
                                    ctypes.POINTER(ctypes.c_double)]),
    ("fem_p1_pattern", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, c_int64_p, c_int64_p, c_void_pp,
                                      c_void_pp]),
    ("fem_p1_assemble", ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 4),
    ("fem_p1_load", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    ("fem_p1_dirichlet", ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 3),
    ("fem_p1_grad_error", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                         ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    ("fem_rt_majorant_rhs", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                           ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]),
    ("fem_majorant_terms", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    ("fem_status_query", ctypes.c_int, [ctypes.c_void_p]),
    ("fem_mesh_destroy", None, [ctypes.c_void_p]),
    ("fem_batch_create", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, c_void_pp]),
    ("fem_batch_bind", ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 5),
    ("fem_batch_tune", ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_void_p]),
    ("fem_batch_config", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                        c_int64_p, ctypes.POINTER(ctypes.c_int)]),
    ("fem_batch_set_config", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    ("fem_batch_assemble", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("fem_batch_graph_launch", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("fem_batch_destroy", None, [ctypes.c_void_p]),
    ("fem_last_error", ctypes.c_char_p, []),
    ("fem_version", ctypes.c_char_p, []),
]

_LIB = None


class FemError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib():
    """The loaded libfem (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise FemError(-1, "load", f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1409_4618_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def check(status: int, where: str):
    if status != 0:
        raise FemError(status, where, lib().fem_last_error().decode())


_HIP = None


def hip():
    """The HIP runtime (for device <-> device/host copies of borrowed pointers)."""
    global _HIP
    if _HIP is None:
        for name in ("libamdhip64.so", "libamdhip64.so.7", "libamdhip64.so.6"):
            try:
                _HIP = ctypes.CDLL(name)
                break
            except OSError:
                continue
        if _HIP is None:
            raise FemError(-1, "load", "libamdhip64.so not found")
        _HIP.hipMemcpyAsync.restype = ctypes.c_int
        _HIP.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                        ctypes.c_void_p]
    return _HIP
