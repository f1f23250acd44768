"""GPU parity of the forward path against the CPU oracle, through the C ABI.

Small and medium meshes (several row tiles plus a ragged tail): topology and
CSR pattern bit-exact, values within relative Frobenius 1e-12, bitwise
symmetric and deterministic. Meshes are relabelled and their element vertex
orders shuffled so every orientation case of Section 2.3 occurs.
"""
import zlib

import numpy as np
import pytest

import meshgen as mg
import oracle
from gpu_util import TOL, dev_tensors, rel_fro, relabel, say

pytestmark = pytest.mark.gpu


def run_case(name, nodes, elems, kind, a=None, b=None):
    import paper_1409_4618_amd as fem
    say(f"[gpu] {name}: kind={kind} T={elems.shape[0]} V={nodes.shape[0]}")
    tn, te, ta, tb = dev_tensors(nodes, elems, a, b)
    mesh = fem.Mesh(tn, te)
    K, M = fem.assemble(mesh, kind, tn, ta, tb)
    rowptr, colind = mesh.pattern(kind)
    topo_g = {k: v.cpu().numpy() for k, v in mesh.topology().items()}
    # a named subset is the same copy of those arrays; an unknown name is refused
    sub = mesh.topology(("signs_e", "edges2nodes"))
    assert list(sub) == ["signs_e", "edges2nodes"]
    assert all(np.array_equal(v.cpu().numpy(), topo_g[k]) for k, v in sub.items())
    with pytest.raises(ValueError):
        mesh.topology(("faces2nodes",) if mesh.dim == 2 else ("edges",))
    K2, M2 = fem.assemble(mesh, kind, tn, ta, tb)
    mesh.status()
    out = dict(mesh=mesh, K=K.cpu().numpy(), M=M.cpu().numpy(), K2=K2.cpu().numpy(),
               M2=M2.cpu().numpy(), rowptr=rowptr.cpu().numpy(), colind=colind.cpu().numpy(),
               topo=topo_g)
    return out


def check_against_oracle(g, nodes, elems, kind, a, b):
    csr, topo = oracle.assemble(nodes, elems, kind, a=a, b=b)
    t = g["topo"]
    assert np.array_equal(t["edges2nodes"], topo.edges2nodes)
    assert np.array_equal(t["elems2edges"], topo.elems2edges)
    assert np.array_equal(t["signs_e"], topo.signs_e)
    if topo.dim == 3:
        assert np.array_equal(t["faces2nodes"], topo.faces2nodes)
        assert np.array_equal(t["elems2faces"], topo.elems2faces)
        assert np.array_equal(t["signs_f"], topo.signs_f)
    assert np.array_equal(g["rowptr"], csr.rowptr)
    assert np.array_equal(g["colind"], csr.colind)
    eK, eM = rel_fro(g["K"], csr.Kv), rel_fro(g["M"], csr.Mv)
    say(f"    rel err K={eK:.2e} M={eM:.2e}")
    assert eK <= TOL and eM <= TOL
    # deterministic: a second launch is bitwise identical
    assert np.array_equal(g["K"], g["K2"]) and np.array_equal(g["M"], g["M2"])
    # bitwise symmetric
    import scipy.sparse as sp
    n = csr.n_rows
    for v in (g["K"], g["M"]):
        A = sp.csr_matrix((v, g["colind"], g["rowptr"]), shape=(n, n))
        D = (A - A.T).tocoo()
        assert np.all(D.data == 0.0)


CASES = [
    ("square 9x7 relabelled", lambda: relabel(*mg.unit_square(9, 7), 1), "ned"),
    ("square 9x7 relabelled", lambda: relabel(*mg.unit_square(9, 7), 1), "rt"),
    ("L-shape m=8", lambda: mg.l_shape(8), "ned"),
    ("kuhn 7x6x5 relabelled", lambda: relabel(*mg.kuhn_box(7, 6, 5), 2), "ned"),
    ("kuhn 7x6x5 relabelled", lambda: relabel(*mg.kuhn_box(7, 6, 5), 2), "rt"),
    ("kuhn 12^3", lambda: mg.kuhn_box(12), "ned"),
    ("kuhn 12^3", lambda: mg.kuhn_box(12), "rt"),
    # relabelled nodes spread each tile's node ids over the whole range
    # (more than 2^16 apart), so no tile sees nearby ids
    ("kuhn strip 16500x1x1 relabelled", lambda: relabel(*mg.kuhn_box(16500, 1, 1, lx=16500.0), 3), "ned"),
    ("kuhn strip 16500x1x1 relabelled", lambda: relabel(*mg.kuhn_box(16500, 1, 1, lx=16500.0), 3), "rt"),
    ("kuhn 1x1x1", lambda: mg.kuhn_box(1), "ned"),
    ("single tet", lambda: (mg.kuhn_box(1)[0], mg.kuhn_box(1)[1][:1]), "rt"),
    ("single triangle", lambda: (np.array([[0., 0.], [1., 0.], [0., 1.]]), np.array([[0, 1, 2]], np.int32)), "ned"),
]


@pytest.mark.parametrize("name,maker,kind", CASES, ids=[f"{c[0]}-{c[2]}" for c in CASES])
def test_forward_matches_oracle(name, maker, kind):
    nodes, elems = maker()
    nodes = np.array(nodes, dtype=np.float64)
    used = np.unique(elems)
    if used.size != nodes.shape[0]:  # drop unused nodes (single-element cases)
        remap = -np.ones(nodes.shape[0], dtype=np.int64)
        remap[used] = np.arange(used.size)
        nodes = nodes[used]
        elems = remap[elems].astype(np.int32)
    rng = np.random.default_rng(zlib.crc32((name + kind).encode()))
    h = 1.0 / max(8, int(round(elems.shape[0] ** (1 / nodes.shape[1]))))
    nodes = mg.perturb_interior(nodes, h, 0.2, rng)
    a = rng.lognormal(0, 0.5, elems.shape[0])
    b = rng.uniform(0.5, 2.0, elems.shape[0])
    g = run_case(name, nodes, elems, kind, a, b)
    check_against_oracle(g, nodes, elems, kind, a, b)


def test_unit_coefficients_equal_null_pointers():
    import torch
    import paper_1409_4618_amd as fem
    nodes, elems = mg.unit_square(32)
    say("[gpu] unit coefficients vs NULL on the 32x32 square")
    tn, te, _, _ = dev_tensors(nodes, elems)
    mesh = fem.Mesh(tn, te)
    ones = torch.ones(elems.shape[0], dtype=torch.float64, device=tn.device)
    K1, M1 = fem.assemble(mesh, "ned", tn, None, None)
    K2, M2 = fem.assemble(mesh, "ned", tn, ones, ones)
    assert torch.equal(K1, K2) and torch.equal(M1, M2)
    # 2D Raviart-Thomas and Nedelec matrices are the same
    K3, M3 = fem.assemble(mesh, "rt", tn, None, None)
    assert torch.equal(K1, K3) and torch.equal(M1, M3)


def test_error_codes():
    import torch
    import paper_1409_4618_amd as fem
    from paper_1409_4618_amd import FemError
    nodes, elems = mg.kuhn_box(2)
    say("[gpu] error codes: range, degenerate, non-finite")
    bad = elems.copy()
    bad[3, 2] = nodes.shape[0]          # node id out of range
    tn, te, _, _ = dev_tensors(nodes, bad)
    with pytest.raises(FemError) as ei:
        fem.Mesh(tn, te)
    assert ei.value.status == 2
    bad = elems.copy()
    bad[5, 1] = bad[5, 0]               # repeated node -> det 0
    tn, te, _, _ = dev_tensors(nodes, bad)
    with pytest.raises(FemError) as ei:
        fem.Mesh(tn, te)
    assert ei.value.status == 3
    n2 = nodes.copy()
    n2[4, 1] = np.nan
    tn, te, _, _ = dev_tensors(n2, elems)
    with pytest.raises(FemError) as ei:
        fem.Mesh(tn, te)
    assert ei.value.status == 4
    # pattern not built -> FEM_ENOTREADY from the C ABI
    tn, te, _, _ = dev_tensors(nodes, elems)
    mesh = fem.Mesh(tn, te)
    from paper_1409_4618_amd._lib import lib
    K = torch.empty(10, dtype=torch.float64, device=tn.device)
    import ctypes
    st = lib().fem_assemble(mesh.handle, 0, ctypes.c_void_p(tn.data_ptr()), None, None,
                            ctypes.c_void_p(K.data_ptr()), None, None)
    assert st == 8
    # a degenerate element introduced after the topology: flagged asynchronously
    fem.assemble(mesh, "ned", tn)
    mesh.status()
    n3 = torch.tensor(nodes, device=tn.device)
    n3[elems[0]] = n3[int(elems[0][0])].clone()   # collapse element 0 onto one point
    fem.assemble(mesh, "ned", n3)
    with pytest.raises(FemError) as ei:
        mesh.status()
    assert ei.value.status == 3
    mesh.status()                       # the error word was cleared


def fan_mesh(axes, n_rim):
    """Tetrahedra fanned around the edges (0, a) for a = 1..axes: n_rim tets per
    axis edge, each (0, a, r_i, r_{i+1}) with the rim r closed into a ring. Row
    (0, a) then has 1 + 3 n_rim entries and n_rim elements."""
    nodes = [[0.0, 0.0, 0.0]]
    dirs = np.array([[1.0, 0.1, 0.2], [0.1, 1.0, 0.3], [0.2, 0.3, 1.0], [-1.0, 0.2, 0.1]])[:axes]
    for d in dirs:
        nodes.append(list(d / np.linalg.norm(d)))
    elems = []
    for a, d in enumerate(dirs, start=1):
        d = d / np.linalg.norm(d)
        u = np.cross(d, [0.3, -0.5, 0.8])
        u /= np.linalg.norm(u)
        w = np.cross(d, u)
        base = len(nodes)
        for i in range(n_rim):
            t = 2 * np.pi * i / n_rim
            nodes.append(list(0.5 * d + np.cos(t) * u + np.sin(t) * w))
        for i in range(n_rim):
            elems.append([0, a, base + i, base + (i + 1) % n_rim])
    return np.array(nodes), np.array(elems, dtype=np.int32)


@pytest.mark.parametrize("kind", ["ned", "rt"])
def test_dense_fans_take_the_row_kernel(kind):
    """Four 84-tet fans around the edges (0, 1) .. (0, 4). Nedelec: those edges
    are the first four rows, so no element-major tile of 4 or more rows fits 256
    lanes and the mesh is assembled by the row kernel; row (0, a) has 253
    entries (near the 255 limit). Raviart-Thomas: the same mesh through the
    element-major kernel (face rows of at most 7 entries)."""
    nodes, elems = fan_mesh(4, 84)
    rng = np.random.default_rng(31)
    a = rng.uniform(0.5, 2.0, elems.shape[0])
    b = rng.uniform(0.5, 2.0, elems.shape[0])
    g = run_case(f"fans 4x84 {kind}", nodes, elems, kind, a, b)
    check_against_oracle(g, nodes, elems, kind, a, b)
    if kind == "ned":
        assert int(np.diff(g["rowptr"]).max()) == 253


def test_row_longer_than_255_is_rejected():
    import paper_1409_4618_amd as fem
    from paper_1409_4618_amd import FemError
    nodes, elems = fan_mesh(1, 86)      # row (0, 1): 1 + 3 * 86 = 259 entries
    say("[gpu] row length 259 -> FEM_EOVERFLOW")
    tn, te, _, _ = dev_tensors(nodes, elems)
    mesh = fem.Mesh(tn, te)
    with pytest.raises(FemError) as ei:
        mesh.pattern("ned")
    assert ei.value.status == 5


def nonconforming_cases():
    """Meshes outside the element-major tiles' assumption (at most two elements
    per facet, no duplicated element): a Kuhn 2^3 box with one tetrahedron
    duplicated (its opposite-edge entries then have two contributions), a 3x3
    square with one triangle duplicated, and three triangles on one edge."""
    n3, e3 = mg.kuhn_box(2)
    n2, e2 = mg.unit_square(3, 3)
    nb = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [0.5, -1.0], [1.2, 1.1]])
    eb = np.array([[0, 1, 2], [0, 1, 3], [1, 0, 4]], np.int32)
    # forty triangles on one edge: its row has 1 + 2 * 40 = 81 entries, beyond
    # the 6-bit column offsets of the element-major records
    nf = np.concatenate([[[0.0, 0.0], [1.0, 0.0]],
                         [[0.5 + 0.4 * np.cos(t), 0.3 + 0.9 * np.sin(t)] for t in np.linspace(0.2, 6.0, 40)]])
    ef = np.array([[0, 1, 2 + i] for i in range(40)], np.int32)
    return [("kuhn 2^3 + duplicated tet", n3, np.concatenate([e3, e3[5:6]]).astype(np.int32), "ned"),
            ("kuhn 2^3 + duplicated tet", n3, np.concatenate([e3, e3[5:6]]).astype(np.int32), "rt"),
            ("square 3x3 + duplicated triangle", n2, np.concatenate([e2, e2[4:5]]).astype(np.int32), "ned"),
            ("three triangles on one edge", nb, eb, "rt"),
            ("forty triangles on one edge", nf, ef, "rt")]


@pytest.mark.parametrize("idx", range(5))
def test_nonconforming_meshes_take_the_row_kernel(idx):
    name, nodes, elems, kind = nonconforming_cases()[idx]
    rng = np.random.default_rng(61 + idx)
    a = rng.uniform(0.5, 2.0, elems.shape[0])
    b = rng.uniform(0.5, 2.0, elems.shape[0])
    g = run_case(name, nodes, elems, kind, a, b)
    check_against_oracle(g, nodes, elems, kind, a, b)


def test_batch_with_a_nonconforming_mesh():
    """Element-major tiling is refused for a batch holding a non-conforming
    mesh; the row tiling gives the single launches' values."""
    import torch
    import paper_1409_4618_amd as fem
    from paper_1409_4618_amd import FemError
    name, nodes, elems, kind = nonconforming_cases()[0]
    ok_nodes, ok_elems = mg.kuhn_box(3)
    meshes, kinds, tn_l, K_l, M_l, ref = [], [], [], [], [], []
    for nd, el in ((nodes, elems), (ok_nodes, ok_elems)):
        tn, te, _, _ = dev_tensors(nd, el)
        m = fem.Mesh(tn, te)
        K, M = fem.assemble(m, kind, tn)
        ref.append((K.clone(), M.clone()))
        meshes.append(m)
        kinds.append(kind)
        tn_l.append(tn)
        K_l.append(torch.zeros_like(K))
        M_l.append(torch.zeros_like(M))
    B = fem.Batch(meshes, kinds)
    B.bind(tn_l, [None, None], [None, None], K_l, M_l)
    with pytest.raises(FemError):
        B.set_config(0, 0)
    B.set_config(128, 0)
    B.assemble()
    for m in meshes:
        m.status()
    for (K, M), K2, M2 in zip(ref, K_l, M_l):
        assert torch.equal(K, K2) and torch.equal(M, M2)


@pytest.mark.parametrize("chunk", ["1", "333"])
@pytest.mark.parametrize("name,maker,kind", [CASES[0], CASES[1], CASES[3], CASES[4]],
                         ids=[f"{c[0]}-{c[2]}" for c in (CASES[0], CASES[1], CASES[3], CASES[4])])
def test_pattern_in_row_chunks_matches_oracle(monkeypatch, chunk, name, maker, kind):
    """The pattern sorted in chunks of whole rows (at most FEM_PAIR_CHUNK pairs,
    a single row alone when it is larger) is the same bit for bit: rowptr,
    colind, and the assembled values that go through the column offsets."""
    monkeypatch.setenv("FEM_PAIR_CHUNK", chunk)
    nodes, elems = maker()
    nodes = np.array(nodes, dtype=np.float64)
    rng = np.random.default_rng(zlib.crc32((name + kind + chunk).encode()))
    nodes = mg.perturb_interior(nodes, 0.05, 0.2, rng)
    a = rng.lognormal(0, 0.5, elems.shape[0])
    b = rng.uniform(0.5, 2.0, elems.shape[0])
    g = run_case(f"{name}, pair chunks of {chunk}", nodes, elems, kind, a, b)
    check_against_oracle(g, nodes, elems, kind, a, b)
