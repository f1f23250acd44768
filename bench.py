"""Benchmark of the GPU assembly path (one JSON line on stdout).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]

Headline (``value``): M tets/s of one numeric assembly of 3D Nedelec K and M in
CSR form (fem_assemble, one kernel launch) on the Kuhn 64^3 workload (1,572,864
tets, interior nodes perturbed by <= 0.2h, a, b ~ lognormal(0, 0.5)), inputs
resident in HBM, topology and pattern built beforehand (as the paper's assembly
routines take precomputed topology). Each timed step first reads a 1 GiB
buffer, so the 256 MB last-level cache holds none of the step's data, then
times one launch with HIP events; ``value`` uses the median. The warm rate
(back-to-back launches, whose inputs partly stay in that cache) is reported
beside it. The same line reports the 128^3 target mesh (with its own roofline
block), the forward + adjoint rate on 96^3 through torch.autograd, the batched
persistent launch on 256 uneven meshes, the one-time topology and pattern
times, and the CPU oracle's rate on a bounded sample, one thread and all host
cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "M tets/s for 3D Nédélec K+M CSR assembly; batched and fwd+bwd vs plain"
PEAK_HBM_GBS = 8000.0


# rocprofv3 summary of the headline kernel (FETCH_SIZE / WRITE_SIZE passes,
# calibrated with a 1 GiB device copy); its traffic figure is reported only
# while the kernel sources, and the tile builder that sizes the tiles, still
# hash to the value it was measured with.
PROFILE = os.path.join(ROOT, "profiles", "fem_forward_ema_ned3d_kuhn64.txt")
PROFILE_128 = os.path.join(ROOT, "profiles", "fem_forward_ema_ned3d_kuhn128.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1409_4618_amd", "csrc", f)
                  for f in ("assemble.hip", "element.h", "fem_internal.h", "topology.hip")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(path=PROFILE):
    """HBM bytes per launch from a committed profile, or None if the kernel
    sources changed since it was taken (or there is no profile)."""
    try:
        with open(path) as fh:
            fields = dict(line.split(":", 1) for line in fh if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    sha = fields.get("kernel_source_sha256", "").strip()
    if not sha or sha != kernel_sources_sha256():
        return None
    try:
        return int(float(fields["traffic_bytes_per_launch"].split()[0]))
    except (KeyError, ValueError):
        return None


def algorithmic_bytes(T, V, dim, nnz, with_coeffs=True):
    """Compulsory bytes of one assembly: read elems, coordinates (each node once)
    and the coefficients; write K and M values once."""
    return T * (dim + 1) * 4 + V * dim * 8 + (16 * T if with_coeffs else 0) + 16 * nnz


def adjoint_bytes(T, V, dim, n_dofs):
    """Compulsory bytes of the quadratic-form adjoint: read elems, coordinates
    (each node once), a, b and u (each dof once); write dL/da and dL/db. The
    vertex derivatives are written by the node sum, not counted here."""
    return T * (dim + 1) * 4 + V * dim * 8 + 16 * T + 8 * n_dofs + 16 * T


def timed(fn, steps, warmup, sync_each=False):
    """Average ms per call of fn() on the current stream, HIP events around the
    timed region, synchronised on both sides."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def setup_mesh(p):
    import torch
    import paper_1409_4618_amd as fem
    d = torch.device("cuda:0")
    tn = torch.tensor(p.nodes, device=d)
    te = torch.tensor(p.elems, device=d)
    ta = None if p.a is None else torch.tensor(p.a, device=d)
    tb = None if p.b is None else torch.tensor(p.b, device=d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mesh = fem.Mesh(tn, te)
    t1 = time.perf_counter()
    n_rows, nnz = mesh.pattern_info(p.kind)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    K = torch.empty(nnz, dtype=torch.float64, device=d)
    M = torch.empty(nnz, dtype=torch.float64, device=d)
    return dict(mesh=mesh, nodes=tn, elems=te, a=ta, b=tb, K=K, M=M, nnz=nnz, n_rows=n_rows,
                t_topology=t1 - t0, t_pattern=t2 - t1)


def forward_rate(p, s, steps, warmup):
    import paper_1409_4618_amd as fem
    run = lambda: fem.assemble_into(s["mesh"], p.kind, s["nodes"], s["a"], s["b"], s["K"], s["M"])
    ms = timed(run, steps, warmup)
    s["mesh"].status()
    T, V = p.T, p.nodes.shape[0]
    bytes_ = algorithmic_bytes(T, V, p.dim, s["nnz"], p.a is not None)
    gbs = bytes_ / (ms * 1e-3) / 1e9
    return dict(ms=ms, mtets=T / (ms * 1e-3) / 1e6, bytes=bytes_, gbs=gbs, frac=gbs / PEAK_HBM_GBS)


class Flush:
    """Evicts the last-level cache by reading a 1 GiB buffer (a read leaves no
    dirty lines to be written back during the timed launch)."""

    def __init__(self):
        import torch
        self.buf = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        self.out = torch.empty((), dtype=torch.float64, device="cuda:0")

    def __call__(self):
        import torch
        torch.sum(self.buf, dim=0, out=self.out)


def cold_times(fn, steps, warmup, flush):
    """Per-step times (ms) of fn(), each after a cache flush: HIP events on the
    current stream around fn() alone; the flush runs before the first event."""
    import torch
    for _ in range(warmup):
        flush()
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for e0, e1 in ev:
        flush()
        e0.record()
        fn()
        e1.record()
    torch.cuda.synchronize()
    return [e0.elapsed_time(e1) for e0, e1 in ev]


def cold_forward(p, s, steps, warmup, flush):
    import paper_1409_4618_amd as fem
    run = lambda: fem.assemble_into(s["mesh"], p.kind, s["nodes"], s["a"], s["b"], s["K"], s["M"])
    times = cold_times(run, steps, warmup, flush)
    s["mesh"].status()
    T, V = p.T, p.nodes.shape[0]
    bytes_ = algorithmic_bytes(T, V, p.dim, s["nnz"], p.a is not None)
    ms = float(np.median(times))
    gbs = bytes_ / (ms * 1e-3) / 1e9
    return dict(ms=ms, ms_min=float(np.min(times)), ms_max=float(np.max(times)),
                mtets=T / (ms * 1e-3) / 1e6, bytes=bytes_, gbs=gbs, frac=gbs / PEAK_HBM_GBS)


def fwd_bwd_rate(p, steps, warmup):
    """Forward + backward through torch.autograd: K, M, L = assemble_quadratic
    (fem_assemble, then fem_quadratic_value_adjoint: L with dL/da, dL/db,
    dL/dnodes from one pass, since the inputs need gradients) and L.backward()
    (the upstream factor applied to those derivatives), timed with HIP events
    around each half of every step. Also reported: the adjoint kernels alone
    (fem_assemble_backward_quadratic), and the adjoint with materialised
    weights gK = gM = u_row u_col."""
    import torch
    import paper_1409_4618_amd as fem
    s = setup_mesh(p)
    d = torch.device("cuda:0")
    rowptr, colind = s["mesh"].pattern(p.kind)
    u = torch.tensor(p.u, device=d)
    x = s["nodes"].clone().requires_grad_(True)
    a = s["a"].clone().requires_grad_(True)
    b = s["b"].clone().requires_grad_(True)
    fwd = forward_rate(p, s, steps, warmup)

    def step(ev=None):
        x.grad = a.grad = b.grad = None
        if ev:
            ev[0].record()
        K, M, L = fem.assemble_quadratic(s["mesh"], p.kind, x, a, b, u)
        if ev:
            ev[1].record()
        L.backward()
        if ev:
            ev[2].record()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(steps)]
    t0 = time.perf_counter()
    for ev in evs:
        step(ev)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / steps
    f_ms = float(np.median([e[0].elapsed_time(e[1]) for e in evs]))
    b_ms = float(np.median([e[1].elapsed_time(e[2]) for e in evs]))
    fb_ms = float(np.median([e[0].elapsed_time(e[2]) for e in evs]))
    s["mesh"].status()

    rows = torch.repeat_interleave(torch.arange(rowptr.numel() - 1, device=d), torch.diff(rowptr))
    w = u[rows] * u[colind.long()]
    del rows
    gn = torch.empty_like(s["nodes"])
    ga = torch.empty(p.T, dtype=torch.float64, device=d)
    gb = torch.empty_like(ga)
    from paper_1409_4618_amd import _ptr, _stream_ptr, check, lib, kind_code
    kc = kind_code(p.kind)

    def bwd_kernels():
        check(lib().fem_assemble_backward_quadratic(s["mesh"].handle, kc, _ptr(s["nodes"]), _ptr(s["a"]),
                                                    _ptr(s["b"]), _ptr(u), _ptr(ga), _ptr(gb), _ptr(gn),
                                                    _stream_ptr()), "fem_assemble_backward_quadratic")

    def bwd_general():
        check(lib().fem_assemble_backward(s["mesh"].handle, kc, _ptr(s["nodes"]), _ptr(s["a"]), _ptr(s["b"]),
                                          _ptr(w), _ptr(w), _ptr(ga), _ptr(gb), _ptr(gn), _stream_ptr()),
              "fem_assemble_backward")

    ms_bk = timed(bwd_kernels, steps, warmup)
    ms_bg = timed(bwd_general, steps, warmup)
    s["mesh"].status()
    out = dict(workload=f"kuhn96_ned3d: {p.T} tets, L = u^T(K(a)+M(b))u through torch.autograd: "
                        "K, M, L = fem.assemble_quadratic(...) (assembly, then L and its adjoint in one pass), "
                        "L.backward() (grads wrt a, b, nodes); "
                        "bwd_kernel_ms: the adjoint kernels alone; bwd_general_ms: the adjoint with "
                        "materialised weights gK = gM = u_row u_col",
               fwd_ms=f_ms, bwd_ms=b_ms, fwd_bwd_ms=fb_ms, fwd_bwd_wall_ms=wall_ms,
               plain_fwd_ms=fwd["ms"], bwd_kernel_ms=ms_bk, bwd_general_ms=ms_bg,
               plain_fwd_mtets=fwd["mtets"], fwd_bwd_mtets=p.T / (fb_ms * 1e-3) / 1e6)
    out["fwd_bwd_over_fwd"] = out["fwd_bwd_mtets"] / out["plain_fwd_mtets"]
    nb = adjoint_bytes(p.T, int(p.nodes.shape[0]), p.dim, int(rowptr.numel() - 1))
    out["bwd_bytes"] = nb
    out["bwd_kernel_gbs"] = nb / (ms_bk * 1e-3) / 1e9
    out["bwd_kernel_frac"] = out["bwd_kernel_gbs"] / PEAK_HBM_GBS
    return out


def small_mesh_latency(steps, warmup):
    """The 2D 32x32 unit square (2,048 triangles, unit coefficients): launch-bound,
    so reported as microseconds per assembly: direct launch, fem_assemble
    captured in a HIP graph (one assembly per replay, and 16 per replay), and
    the one-mesh persistent batch kernel's graph."""
    import torch
    import meshgen as mg
    import paper_1409_4618_amd as fem
    p = mg.square_ned32()
    s = setup_mesh(p)
    run = lambda: fem.assemble_into(s["mesh"], p.kind, s["nodes"], None, None, s["K"], s["M"])
    us_direct = timed(run, steps, warmup) * 1e3

    def capture(n):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            run()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(n):
                run()
        torch.cuda.synchronize()
        return g

    g1, g16 = capture(1), capture(16)
    us_graph = timed(g1.replay, steps, warmup) * 1e3
    us_graph16 = timed(g16.replay, steps, warmup) * 1e3 / 16
    B = fem.Batch([s["mesh"]], [p.kind])
    B.bind([s["nodes"]], [None], [None], [s["K"]], [s["M"]])
    us_batch = timed(B.graph_launch, steps, warmup) * 1e3
    s["mesh"].status()
    return {"workload": "square32_ned2d: 2D Nedelec K+M, unit square 32x32 (2,048 triangles), unit coefficients",
            "us_direct": us_direct, "us_graph": us_graph, "us_graph_x16_per_assembly": us_graph16,
            "us_batch_kernel_graph": us_batch, "nnz": s["nnz"],
            "note": "us_graph: fem_assemble captured in a HIP graph (torch.cuda.CUDAGraph), one replay per "
                    "assembly; us_graph_x16_per_assembly: 16 assemblies captured in one graph; "
                    "us_batch_kernel_graph: a one-mesh batch's graph (its default configuration: one grid launch "
                    "for the mesh's element kind)"}


def batched_rate(steps, warmup, ref_mtets, scale=1.0):
    import torch
    import meshgen as mg
    import paper_1409_4618_amd as fem
    probs = mg.batch_problems(seed=4, count=256, scale=scale)
    d = torch.device("cuda:0")
    meshes, kinds, nodes, a, b, Ks, Ms = [], [], [], [], [], [], []
    for p in probs:
        tn = torch.tensor(p.nodes, device=d)
        m = fem.Mesh(tn, torch.tensor(p.elems, device=d))
        _, nnz = m.pattern_info(p.kind)
        meshes.append(m)
        kinds.append(p.kind)
        nodes.append(tn)
        a.append(torch.tensor(p.a, device=d))
        b.append(torch.tensor(p.b, device=d))
        Ks.append(torch.empty(nnz, dtype=torch.float64, device=d))
        Ms.append(torch.empty(nnz, dtype=torch.float64, device=d))
    T_total = sum(p.T for p in probs)
    bytes_total = sum(algorithmic_bytes(p.T, int(p.nodes.shape[0]), p.dim, int(K.numel()), p.a is not None)
                      for p, K in zip(probs, Ks))
    B = fem.Batch(meshes, kinds)
    B.bind(nodes, a, b, Ks, Ms)
    # the autotuner's JSON-lines cache (FEM_TUNE_CACHE overrides the location)
    cache = os.environ.get("FEM_TUNE_CACHE", os.path.join(tempfile.gettempdir(), "fem_batch_tune.jsonl"))
    B.tune(cache)
    cfg = B.config()
    ms_graph = timed(B.graph_launch, steps, warmup)
    ms_direct = timed(B.assemble, steps, warmup)

    def sequential():
        for i in range(len(meshes)):
            fem.assemble_into(meshes[i], kinds[i], nodes[i], a[i], b[i], Ks[i], Ms[i])

    ms_seq = timed(sequential, max(1, steps // 2), 1)
    for m in meshes:
        m.status()
    mt = T_total / (ms_graph * 1e-3) / 1e6
    return dict(workload=f"256 meshes (2D/3D, Nedelec/RT), {T_total} elements",
                elements=T_total, ms_graph=ms_graph, ms_direct=ms_direct, ms_sequential=ms_seq,
                mtets=mt, sequential_mtets=T_total / (ms_seq * 1e-3) / 1e6,
                over_plain_forward=mt / ref_mtets if ref_mtets else None, over_sequential=ms_seq / ms_graph,
                tuned=cfg,
                bytes=bytes_total, achieved_gbs=bytes_total / (ms_graph * 1e-3) / 1e9,
                frac=bytes_total / (ms_graph * 1e-3) / 1e9 / PEAK_HBM_GBS)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_chunk(args):
    """Worker of the all-cores baseline: the oracle's numeric phase on one
    contiguous chunk of elements, repeated for about ``seconds``; returns
    (elements done, start, end) in wall-clock seconds."""
    nodes, elems, kind, a, b, seconds = args
    from threadpoolctl import threadpool_limits
    import oracle
    topo = oracle.build_topology(elems, nodes.shape[0])
    with threadpool_limits(limits=1):
        t0 = time.time()
        done = 0
        while True:
            oracle.assemble(nodes, elems, kind, a=a, b=b, topo=topo)
            done += elems.shape[0]
            if time.time() - t0 >= seconds:
                break
        return done, t0, time.time()


def cpu_baseline(p, target_seconds=12.0, workers=None):
    """The oracle (numeric phase: quadrature local matrices + CSR accumulation,
    topology given) on a bounded sample of the same mesh: one thread on the
    first 100k tets, and all host cores (at most 16 worker processes, each on
    its own 100k-tet chunk) at once."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import oracle
    from threadpoolctl import threadpool_limits
    n = 100000
    elems = p.elems[:n]
    topo = oracle.build_topology(elems, p.nodes.shape[0])
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        oracle.assemble(p.nodes, elems, p.kind, a=p.a[:n], b=p.b[:n], topo=topo)
        dt = time.perf_counter() - t0
        reps = max(1, int(target_seconds / max(dt, 1e-3)))
        t0 = time.perf_counter()
        for _ in range(reps):
            oracle.assemble(p.nodes, elems, p.kind, a=p.a[:n], b=p.b[:n], topo=topo)
        dt = (time.perf_counter() - t0) / reps
    single = n / dt / 1e6
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    nw = workers or max(1, min(16, avail))
    jobs = []
    for w in range(nw):
        lo = (w * n) % max(1, p.T - n)
        e = p.elems[lo:lo + n]
        jobs.append((p.nodes, e, p.kind, p.a[lo:lo + n], p.b[lo:lo + n], target_seconds))
    with cf.ProcessPoolExecutor(max_workers=nw, mp_context=mp.get_context("spawn")) as ex:
        res = list(ex.map(_oracle_chunk, jobs))
    total = sum(r[0] for r in res)
    span = max(r[2] for r in res) - min(r[1] for r in res)
    return {"value": total / span / 1e6, "unit": "M tets/s", "cores": nw, "kind": "oracle",
            "sample": f"{nw} worker processes (one thread each), each repeating the numeric phase "
                      f"(quadrature local matrices + CSR accumulation, topology given) on its own "
                      f"{n}-tet chunk of the same 64^3 mesh for about {target_seconds:.0f} s; "
                      f"rate = all elements done / wall time from the first start to the last end",
            "single_thread": {"value": single, "cores": 1,
                              "sample": f"first {n} tets of the same mesh, {reps} reps, 1 thread"},
            "cpu_count": os.cpu_count(), "cpus_available": avail, "cpu_model": cpu_model()}


# The paper's MATLAB assembly times in seconds (Section 3.3, the 2D L-shape and
# 3D unit-cube timing tables; 64x Xeon E7-8837, R2011b) per level:
# (K_RT, M_RT, K_Ned, M_Ned). Context for the level curves, not a target.
PAPER_3D_S = {1: (0.02, 0.09, 0.05, 0.09), 2: (0.14, 0.39, 0.30, 0.79), 3: (0.82, 2.18, 1.92, 4.53),
              4: (7.15, 15.35, 15.44, 33.43), 5: (59.37, 125.71, 129.91, 282.14),
              6: (503.89, 1054.49, 1125.08, 2291.50), 7: (4437.84, 8717.70, 10232.01, 20028.06)}
PAPER_2D_S = {5: (0.03, 0.06, 0.03, 0.03), 6: (0.11, 0.51, 0.11, 0.47), 7: (0.41, 1.08, 0.40, 1.02),
              8: (1.70, 3.59, 1.82, 3.65), 9: (7.49, 12.82, 7.49, 12.94), 10: (30.89, 52.09, 30.83, 54.86),
              11: (132.95, 216.64, 132.56, 230.44), 12: (597.37, 919.36, 583.86, 931.79),
              13: (2620.11, 3969.16, 2840.51, 4121.33)}


def level_curves(steps, warmup, max_level_3d=7, max_level_2d=13):
    """The paper's timing tables re-run on the GPU: unit coefficients and
    unperturbed meshes (the paper's timing setting), the 3D unit cube at levels
    1-7 (n = 3 2^level cubes per side, 6 tets each; level 7 has 340 M tets and
    6.5 G Nedelec nonzeros per matrix) and the 2D L-shape at levels 5-13 (m =
    2^level cells per half side; level 13 has 3.02 G nonzeros per matrix), both
    kinds, each on a topology handle of its own (so that one kind's pattern and
    tiles are resident at a time). The meshes are laid out on the device. Per
    level and kind: K + M together, K alone and M alone (the paper's columns),
    warm median of `steps` launches each, M elements/s, the fraction of 8 TB/s
    (K + M), the growth from the previous level (the paper prints it: 4 in 2D,
    8 in 3D is optimal), the paper's seconds beside them, and the CPU oracle
    (numeric phase, one thread) at the small levels. The paper's 2D level 14
    has 4.8 G element-edge slots (T times the edges per element), beyond the
    library's int32 slot indices. A level that fails (out of device memory) is
    recorded with its error and the curve goes on."""
    import torch
    import meshgen as mg
    import oracle
    import paper_1409_4618_amd as fem
    from threadpoolctl import threadpool_limits
    d = torch.device("cuda:0")
    out = []
    prev = {}
    cases = ([("cube", L, 3 * 2 ** L) for L in range(1, max_level_3d + 1)] +
             [("lshape", L, 2 ** L) for L in range(5, max_level_2d + 1)])
    for dom, L, n in cases:
        tn, te = mg.kuhn_box_torch(n, d) if dom == "cube" else mg.l_shape_torch(n, d)
        T, dim = int(te.shape[0]), int(te.shape[1]) - 1
        paper = (PAPER_3D_S if dim == 3 else PAPER_2D_S)[L]
        mesh = s = None
        try:
            for kind in ("rt", "ned"):
                mesh = s = None
                torch.cuda.empty_cache()
                mesh = fem.Mesh(tn, te)
                p = mg.Problem(f"{dom}{L}_{kind}", kind, tn, te)
                n_rows, nnz = mesh.pattern_info(kind)
                s = dict(mesh=mesh, nodes=tn, elems=te, a=None, b=None, nnz=nnz, n_rows=n_rows,
                         K=torch.empty(nnz, dtype=torch.float64, device=d),
                         M=torch.empty(nnz, dtype=torch.float64, device=d))
                st, wu = max(5, steps // 10), max(2, warmup // 10)
                f = forward_rate(p, s, st, wu)
                k_ms = timed(lambda: fem.assemble_into(mesh, kind, tn, None, None, s["K"], None), st, wu)
                m_ms = timed(lambda: fem.assemble_into(mesh, kind, tn, None, None, None, s["M"]), st, wu)
                mesh.status()
                pk, pm = (paper[0], paper[1]) if kind == "rt" else (paper[2], paper[3])
                row = {"domain": dom, "level": L, "kind": kind, "elements": T, "rows": n_rows, "nnz": nnz,
                       "ms": round(f["ms"], 5), "k_ms": round(k_ms, 5), "m_ms": round(m_ms, 5),
                       "mel_s": round(f["mtets"], 1), "frac": round(f["frac"], 4),
                       "paper_k_s": pk, "paper_m_s": pm, "paper_mel_s": round(T / (pk + pm) / 1e6, 4)}
                if (dom, kind) in prev:
                    row["growth"] = round(f["ms"] / prev[(dom, kind)], 2)
                prev[(dom, kind)] = f["ms"]
                if T <= 100000:
                    nodes, elems = tn.cpu().numpy(), te.cpu().numpy()
                    with threadpool_limits(limits=1):
                        t0 = time.perf_counter()
                        oracle.assemble(nodes, elems, kind)
                        row["oracle_1thread_mel_s"] = round(T / (time.perf_counter() - t0) / 1e6, 4)
                out.append(row)
            log(f"bench:   {dom} level {L}: {out[-1]['mel_s']} M el/s (ned), {out[-2]['mel_s']} (rt)")
        except (RuntimeError, fem.FemError) as e:
            out.append({"domain": dom, "level": L, "elements": T, "error": str(e)[:200]})
            log(f"bench:   {dom} level {L}: not run ({str(e)[:120]})")
        mesh = s = None
        del tn, te
        torch.cuda.empty_cache()
    return out


def eddy_rate(n=512):
    """The 2D eddy-current example (Section 4.2) on the n x n unit square: the
    whole pipeline (K + M assembly, load vector, Jacobi-CG to a recursive
    residual of 1e-12, energy error), each phase timed with HIP events (one run
    after a warm-up run), against the paper's printed error; and the
    squared L2 norm routine (fem_norm_L2) on the same mesh and on Kuhn 64^3."""
    import torch
    import meshgen as mg
    import paper_1409_4618_amd as fem
    d = torch.device("cuda:0")
    nodes, elems = mg.unit_square(n)
    tn = torch.tensor(nodes, device=d)
    te = torch.tensor(elems, device=d)
    mesh = fem.Mesh(tn, te)
    rowptr, colind = mesh.pattern_device("ned")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]

    def run(record):
        if record:
            ev[0].record()
        K, M = fem._assemble_values(mesh, "ned", tn)
        if record:
            ev[1].record()
        f = fem.load_vector(mesh, "ned", tn, fem.FEM_FN_EDDY_F)
        if record:
            ev[2].record()
        v, iters, res = fem.cg_solve(rowptr, colind, K, f, B=M, rtol=1e-12)
        if record:
            ev[3].record()
        _, e2 = fem.field_error(mesh, "ned", tn, v, fem.FEM_FN_EDDY_E, fem.FEM_FN_EDDY_CURL_E)
        if record:
            ev[4].record()
        return iters, res, e2
    run(False)
    torch.cuda.synchronize()
    iters, res, e2 = run(True)
    torch.cuda.synchronize()
    mesh.status()
    ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(4)]
    nnz = colind.numel()
    nrow = rowptr.numel() - 1
    # bytes of one CG iteration: the product reads rowptr, colind, the system's
    # values K + M (formed once per solve) and the gathered z, p (each column
    # value once), writes p and q; the update reads x, p, q, r, 1/diag and
    # writes x, r, z
    it_bytes = 8 * (nrow + 1) + 4 * nnz + 8 * nnz + 16 * nrow + 16 * nrow + 5 * 8 * nrow + 3 * 8 * nrow
    cg_it_ms = ms[2] / max(iters, 1)
    out = {"workload": f"2D eddy current, unit square {n}x{n} ({elems.shape[0]} triangles, {nrow} edges)",
           "error": math.sqrt(e2.item()), "paper_error": {128: 2.358185e-02, 256: 1.179151e-02, 512: 5.895834e-03,
                                                          1024: 2.947927e-03}.get(n),
           "assemble_ms": ms[0], "load_vector_ms": ms[1], "cg_ms": ms[2], "cg_iterations": iters,
           "cg_true_rel_residual": res, "cg_us_per_iteration": 1e3 * cg_it_ms,
           "cg_iteration_gbs": it_bytes / (cg_it_ms * 1e-3) / 1e9, "error_ms": ms[3], "total_ms": sum(ms)}
    # fem_norm_L2 rates
    steps = 20
    ms_l2 = timed(lambda: fem.norm_L2(mesh, tn, fem.FEM_FN_EDDY_E), steps, 3)
    out["norm_L2_eddy_E"] = {"elements": int(elems.shape[0]), "ms": ms_l2, "quad_points": 16,
                             "mel_s": elems.shape[0] / (ms_l2 * 1e-3) / 1e6}
    p = mg.kuhn64_ned()
    t3 = torch.tensor(p.nodes, device=d)
    m3 = fem.Mesh(t3, torch.tensor(p.elems, device=d))
    terms = [1.0, 0, 1, 1, 0, -2.0, 0, 0, 0, 2, 0.5, 1, 2, 0, 1]
    ms3 = timed(lambda: fem.norm_L2(m3, t3, fem.FEM_FN_POLYNOMIAL, terms), steps, 3)
    out["norm_L2_kuhn64_polynomial"] = {"elements": p.T, "ms": ms3, "quad_points": 125,
                                        "mel_s": p.T / (ms3 * 1e-3) / 1e6}
    m3.status()
    return out


def majorant_rate(n2=1024, n3=48):
    """The majorant minimisation of Section 4.1 (Algorithm 1) on the unit square
    (n2 x n2 cells, 2 n2^2 triangles) and the unit cube (Kuhn n3^3): the whole
    run (P1 assembly, load, boundary elimination and CG; per beta iteration the
    RT right-hand side, CG on (1 + beta) C^2 K + (1 + 1/beta) M and the majorant
    terms) timed with HIP events after a warm-up run, and the iterations'
    beta, majorant and efficiency index (2D: against the paper's printed table)."""
    import torch
    import meshgen as mg
    import paper_1409_4618_amd as fem
    from paper_1409_4618_amd.majorant import minimise
    d = torch.device("cuda:0")
    out = {}
    for dim, n in ((2, n2), (3, n3)):
        nodes, elems = mg.unit_square(n) if dim == 2 else mg.kuhn_box(n)
        tn = torch.tensor(nodes, device=d)
        mesh = fem.Mesh(tn, torch.tensor(elems, device=d))
        minimise(mesh, tn)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        r = minimise(mesh, tn)
        e1.record()
        torch.cuda.synchronize()
        out[f"{dim}d"] = {"workload": (f"unit square {n}x{n}" if dim == 2 else f"Kuhn {n}^3") +
                          f" ({elems.shape[0]} elements), bubble solution",
                          "ms": e0.elapsed_time(e1), "error_grad": r["error"],
                          "cg_iterations_v": r["cg_iterations_v"],
                          "iterations": [{"beta": it["beta"], "majorant": it["majorant"], "ieff": it["ieff"],
                                          "cg_iterations": it["cg_iterations"]} for it in r["iterations"]]}
    out["2d"]["paper"] = {1024: [(1.000, 0.000412, 1.73), (3.294, 0.000363, 1.52), (3.294, 0.000363, 1.52)],
                          256: [(1.000, 0.001648, 1.73), (3.294, 0.001453, 1.52), (3.294, 0.001453, 1.52)]}.get(n2)
    return out


def calib_copy():
    """A plain device copy of known size (1 GiB read + 1 GiB written), to scale the
    HBM byte counters of a profiler run."""
    import torch
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return 2 * src.numel() * 8


def stream_ceiling(kernel_ms, traffic):
    """Practical HBM rates of plain streaming kernels (torch's fill, copy and a
    broadcast copy that reads N and writes 2N doubles, about the forward kernel's
    read:write mix), with N = 28 Mi doubles. The forward kernel's measured
    traffic rate is reported beside them when its profile is current."""
    import torch
    n = 28 << 20
    x = torch.rand(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty(2 * n, dtype=torch.float64, device="cuda:0")
    z = torch.empty(n, dtype=torch.float64, device="cuda:0")

    def best_ms(fn, reps=30):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        best = float("inf")
        for _ in range(reps):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    fill = 2 * n * 8 / best_ms(lambda: y.fill_(1.0)) / 1e6
    copy = 2 * n * 8 / best_ms(lambda: z.copy_(x)) / 1e6
    mix = 3 * n * 8 / best_ms(lambda: y.view(n, 2).copy_(x.unsqueeze(1).expand(n, 2))) / 1e6
    del x, y, z
    out = {"unit": "GB/s", "fill": round(fill, 1), "copy": round(copy, 1), "read1_write2": round(mix, 1)}
    if traffic:
        rate = traffic / (kernel_ms * 1e-3) / 1e9
        out["forward_traffic_rate"] = round(rate, 1)
        out["forward_over_read1_write2"] = round(rate / mix, 4)
    return out


PAPER_EDDY_ERRORS = {128: 2.358185e-02, 256: 1.179151e-02, 512: 5.895834e-03, 1024: 2.947927e-03,
                     2048: 1.473965e-03, 4096: 7.369826e-04}


def eddy_table():
    """The paper's eddy-current table re-run on the GPU: the whole pipeline
    (assembly, load vector, Jacobi-CG to a recursive relative residual of 1e-12,
    energy error) on all six unit-square meshes, 128^2 to 4096^2 (50 M edges),
    each error printed to the paper's 7 digits against the printed value. The
    CG reports its progress on stderr every 20,000 iterations (FEM_CG_LOG)."""
    import torch
    import meshgen as mg
    import paper_1409_4618_amd as fem
    from paper_1409_4618_amd.eddy import eddy_current
    d = torch.device("cuda:0")
    os.environ["FEM_CG_LOG"] = "20000"
    rows = []
    for n, printed in PAPER_EDDY_ERRORS.items():
        log(f"bench:   eddy {n}x{n}")
        tn, te = mg.unit_square_torch(n, d)
        mesh = fem.Mesh(tn, te)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = eddy_current(mesh, tn)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        rows.append({"n": n, "triangles": int(te.shape[0]), "edges": mesh.n_edges, "error": f"{out['error']:.9e}",
                     "printed": f"{printed:.6e}", "matches": f"{out['error']:.6e}" == f"{printed:.6e}",
                     "cg_iterations": out["iters"], "cg_true_rel_residual": out["rel_resid"], "seconds": round(sec, 3)})
        log(f"bench:   eddy {n}x{n}: error {out['error']:.9e} (paper {printed:.6e}), {out['iters']} CG iterations, "
            f"{sec:.1f} s")
        del mesh, out, tn, te
        torch.cuda.empty_cache()
    del os.environ["FEM_CG_LOG"]
    return {"eddy_table": rows}


def only_workload(args):
    import meshgen as mg
    if args.only in ("kuhn128_ned3d", "kuhn128_rt3d"):
        p = mg.kuhn128_ned() if args.only == "kuhn128_ned3d" else mg.kuhn128_rt()
        s = setup_mesh(p)
        f = forward_rate(p, s, args.steps, args.warmup)
        out = {"workload": args.only, "ms": f["ms"], "mtets": f["mtets"], "bytes_per_launch": f["bytes"],
               "achieved_gbs": f["gbs"], "frac": f["frac"]}
    elif args.only == "kuhn96_fwd_bwd":
        out = fwd_bwd_rate(mg.kuhn96_ned_grad(), args.steps, args.warmup)
    elif args.only == "eddy":
        out = eddy_rate()
    elif args.only == "eddy_table":
        out = eddy_table()
    elif args.only == "majorant":
        out = majorant_rate()
    elif args.only == "levels":
        out = {"levels": level_curves(args.steps, args.warmup)}
    elif args.only == "small2d":
        out = small_mesh_latency(args.steps, args.warmup)
    else:
        out = batched_rate(args.steps, args.warmup, None)
    if args.calib_copy:
        out["calib_copy_bytes"] = calib_copy()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--quick", action="store_true", help="headline only (for profiling runs)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 1 GiB device copy (profiler byte-counter calibration)")
    ap.add_argument("--only", choices=["kuhn128_ned3d", "kuhn128_rt3d", "kuhn96_fwd_bwd", "batch256", "eddy",
                                       "eddy_table", "majorant", "levels", "small2d"],
                    help="time one secondary workload alone and print its JSON (for profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "libfem assembles on one GPU per process: --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import meshgen as mg
    import paper_1409_4618_amd as fem  # noqa: F401  (fails loudly if libfem.so is missing)
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")

    if args.only:
        print(json.dumps(only_workload(args)), flush=True)
        return

    log("bench: building kuhn64_ned3d")
    p64 = mg.kuhn64_ned()
    s64 = setup_mesh(p64)
    flush = Flush()
    log("bench: timing forward 64^3 (cold: cache flushed before each step)")
    c64 = cold_forward(p64, s64, args.steps, args.warmup, flush)
    log("bench: timing forward 64^3 (warm: back-to-back launches)")
    f64 = forward_rate(p64, s64, args.steps, args.warmup)
    result = {
        "metric": METRIC,
        "value": round(c64["mtets"], 3),
        "unit": "M tets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(c64["ms"], 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "kuhn64_ned3d: 3D Nedelec K+M CSR assembly, Kuhn 64^3 unit cube "
                               "(1,572,864 tets), interior nodes +-0.2h, a,b ~ lognormal(0,0.5), seed 2; "
                               "last-level cache flushed (1 GiB read) before each timed launch, median",
                   "elements": p64.T, "nodes": int(p64.nodes.shape[0]), "nnz": s64["nnz"],
                   "rows": s64["n_rows"]},
        "roofline": {"bound": "hbm", "achieved": round(c64["gbs"], 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(c64["frac"], 4), "traffic": profiled_traffic(),
                     "kernel": "fem::k_forward_ema<2, 256>", "bytes_per_launch": c64["bytes"]},
        "warm": {"ms": round(f64["ms"], 6), "mtets": round(f64["mtets"], 3),
                 "achieved_gbs": round(f64["gbs"], 1), "frac": round(f64["frac"], 4),
                 "note": "back-to-back launches (inputs partly held in the 256 MB last-level cache)"},
        "cold_spread_ms": [round(c64["ms_min"], 6), round(c64["ms_max"], 6)],
    }
    if args.calib_copy:
        result["calib_copy_bytes"] = calib_copy()
    if args.quick:
        print(json.dumps(result), flush=True)
        return
    log("bench: streaming ceilings")
    result["stream_ceiling"] = stream_ceiling(f64["ms"], result["roofline"]["traffic"])
    result["one_time_s"] = {"topology": round(s64["t_topology"], 4), "pattern": round(s64["t_pattern"], 4)}
    del s64
    torch.cuda.empty_cache()

    log("bench: kuhn128_ned3d target")
    p128 = mg.kuhn128_ned()
    s128 = setup_mesh(p128)
    f128 = forward_rate(p128, s128, args.steps, args.warmup)
    c128 = cold_forward(p128, s128, args.steps, args.warmup, flush)
    result["target_128"] = {"workload": "kuhn128_ned3d: 12,582,912 tets, +-0.15h, lognormal a,b, seed 1",
                            "ms": round(f128["ms"], 6), "mtets": round(f128["mtets"], 3),
                            "achieved_gbs": round(f128["gbs"], 1), "frac": round(f128["frac"], 4),
                            "cold_ms": round(c128["ms"], 6), "cold_frac": round(c128["frac"], 4),
                            "roofline": {"bound": "hbm", "achieved": round(f128["gbs"], 1), "peak": PEAK_HBM_GBS,
                                         "unit": "GB/s", "frac": round(f128["frac"], 4),
                                         "traffic": profiled_traffic(PROFILE_128),
                                         "kernel": "fem::k_forward_ema<2, 256>", "bytes_per_launch": f128["bytes"]},
                            "topology_s": round(s128["t_topology"], 4), "pattern_s": round(s128["t_pattern"], 4)}
    del s128
    torch.cuda.empty_cache()

    log("bench: kuhn128_rt3d")
    prt = mg.kuhn128_rt()
    srt = setup_mesh(prt)
    frt = forward_rate(prt, srt, args.steps, args.warmup)
    result["rt_128"] = {"workload": "kuhn128_rt3d: 12,582,912 tets, 3D Raviart-Thomas", "ms": round(frt["ms"], 6),
                        "mtets": round(frt["mtets"], 3), "achieved_gbs": round(frt["gbs"], 1),
                        "frac": round(frt["frac"], 4)}
    del srt
    torch.cuda.empty_cache()

    log("bench: kuhn96 forward + adjoint")
    result["fwd_bwd"] = {k: (round(v, 6) if isinstance(v, float) else v)
                         for k, v in fwd_bwd_rate(mg.kuhn96_ned_grad(), args.steps, args.warmup).items()}
    torch.cuda.empty_cache()

    log("bench: square32 latency")
    result["small_2d"] = {k: (round(v, 3) if isinstance(v, float) else v)
                          for k, v in small_mesh_latency(args.steps, args.warmup).items()}

    log("bench: batched 256 meshes")
    result["batched"] = {k: (round(v, 6) if isinstance(v, float) else v)
                         for k, v in batched_rate(args.steps, args.warmup, f64["mtets"]).items()}
    torch.cuda.empty_cache()

    log("bench: 2D eddy-current pipeline and norm_L2")
    result["eddy_2d"] = {k: (round(v, 6) if isinstance(v, float) and k.endswith("_ms") else v)
                         for k, v in eddy_rate().items()}
    torch.cuda.empty_cache()

    log("bench: majorant minimisation")
    result["majorant"] = majorant_rate()
    torch.cuda.empty_cache()

    log("bench: level curves (paper's timing meshes)")
    result["levels"] = level_curves(args.steps, args.warmup)
    torch.cuda.empty_cache()

    if not args.no_cpu:
        log("bench: CPU oracle baseline")
        result["cpu_baseline"] = cpu_baseline(p64)
    result["paper_context"] = ("MATLAB R2011b on 64x Xeon E7-8837: 3D Nedelec K+M on 96^3-size mesh "
                               "(level 5) 129.91+282.14 s = 0.0129 M tets/s")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
