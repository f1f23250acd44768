"""CPU checks of the C-ABI library: it loads, exports every entry point declared
in include/fem.h, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fem.h")


@pytest.fixture(scope="module")
def L():
    from paper_1409_4618_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1409_4618_amd import build
        build.build()
    return _lib.lib()


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fem_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    syms = declared_symbols()
    for name in ("fem_topology", "fem_pattern", "fem_assemble", "fem_assemble_backward",
                 "fem_batch_create", "fem_batch_bind", "fem_batch_tune", "fem_batch_assemble",
                 "fem_batch_graph_launch", "fem_status_query", "fem_last_error"):
        assert name in syms


def test_library_exports_every_declared_symbol(L):
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_1409_4618_amd import _lib
    bound = {name for name, _, _ in _lib.SIGNATURES}
    assert set(declared_symbols()) == bound


def test_argument_errors_without_gpu(L):
    from paper_1409_4618_amd._lib import FEM_NEDELEC
    out = ctypes.c_void_p()
    # NULL output handle, bad dim, empty mesh, NULL pointers: rejected on the host
    assert L.fem_topology(None, 10, 3, None, 10, None, None) == 1
    assert L.fem_topology(None, 10, 5, None, 10, None, ctypes.byref(out)) == 1
    assert b"dim" in L.fem_last_error()
    assert L.fem_topology(None, 0, 3, None, 10, None, ctypes.byref(out)) == 1
    assert L.fem_topology(None, 10, 3, None, 10, None, ctypes.byref(out)) == 1
    assert out.value is None
    # int32 limits
    assert L.fem_topology(ctypes.c_void_p(16), 1 << 31, 3, ctypes.c_void_p(16), 10, None,
                          ctypes.byref(out)) == 5
    assert L.fem_topology(ctypes.c_void_p(16), 10, 3, ctypes.c_void_p(16), 1 << 29, None,
                          ctypes.byref(out)) == 5
    assert L.fem_topology(ctypes.c_void_p(16), 1 << 30, 3, ctypes.c_void_p(16), 10, None,
                          ctypes.byref(out)) == 5  # n_nodes * dim >= 2^31
    # NULL handles
    assert L.fem_assemble(None, FEM_NEDELEC, None, None, None, None, None, None) == 1
    assert L.fem_assemble_backward(None, FEM_NEDELEC, *([None] * 9)) == 1
    assert L.fem_pattern(None, FEM_NEDELEC, None, None, None, None, None) == 1
    assert L.fem_batch_create(None, None, 0, ctypes.byref(out)) == 1
    assert L.fem_batch_assemble(None, None) == 1
    assert L.fem_status_query(None) == 1
    L.fem_mesh_destroy(None)
    L.fem_batch_destroy(None)
    assert L.fem_version().startswith(b"libfem")


def test_product_path_has_no_cpu_fallback():
    """The package imports no oracle code and no CPU implementation."""
    pkg = os.path.join(ROOT, "paper_1409_4618_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "import oracle" not in src and "from oracle" not in src, fn


def test_missing_library_fails_loudly():
    """Without libfem.so every entry point raises (no silent CPU path): checked
    in a fresh interpreter whose loader points at a file that does not exist."""
    import subprocess
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import paper_1409_4618_amd._lib as L\n"
        "L.LIB_PATH = '/nonexistent/libfem.so'\n"
        "import paper_1409_4618_amd as fem\n"
        "try:\n"
        "    fem.kind_code('ned'); fem.lib()\n"
        "except fem.FemError as e:\n"
        "    print('raised:', e)\n"
        "    sys.exit(0)\n"
        "sys.exit(3)\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "is missing" in r.stdout


def test_checked_build_exports_every_declared_symbol():
    """libfem_check.so (the bounds-checked build) is built beside libfem.so and
    exports the same entry points."""
    from paper_1409_4618_amd import build
    if not os.path.exists(build.LIB_CHECK):
        build.build()
    L = ctypes.CDLL(build.LIB_CHECK)
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing, missing
