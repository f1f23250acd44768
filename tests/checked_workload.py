"""A fixed workload over every kernel family of the library, for the checked
build's test (not a test module): ``run(out_dir)`` runs it with whichever
library the process loaded and saves every result to ``out_dir/results.npz``;
``python checked_workload.py ROOT OUT_DIR`` does the same in a child process
(the test starts it with FEM_CHECK=1, which loads libfem_check.so).

Covered: topology and patterns; the forward (element-major tiles, and the row
kernels when FEM_FWD_PATH=rows) for 2D and 3D, both kinds, relabelled meshes;
the batch (element-major tiles of 256 and 128 lanes, row tiles, the per-kind
launches); the adjoint
(separate and shared weights, the quadratic form, vertex derivatives) and the
quadratic-form value; integration, load vector, H(curl) error and CG of the
eddy example; the P1 system, its boundary elimination and error; the
Raviart-Thomas majorant right-hand side and terms. Every call is followed by
the mesh's status check, which raises if a kernel flagged an index out of
range.
"""
import os
import sys

import numpy as np


def _meshes():
    import meshgen as mg
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from gpu_util import relabel
    rng = np.random.default_rng(77)
    out = []
    n3, e3 = relabel(*mg.kuhn_box(5, 4, 3), 3)
    n3 = mg.perturb_interior(np.asarray(n3, dtype=np.float64), 0.1, 0.2, rng)
    n2, e2 = relabel(*mg.unit_square(9, 7), 4)
    n2 = mg.perturb_interior(np.asarray(n2, dtype=np.float64), 0.05, 0.2, rng)
    for name, nodes, elems in (("k3", n3, e3), ("s2", n2, e2)):
        T = elems.shape[0]
        out.append((name, nodes, np.asarray(elems, np.int32), rng.lognormal(0, 0.5, T), rng.uniform(0.5, 2, T)))
    return out


def run(out_dir):
    import torch
    import meshgen as mg
    import paper_1409_4618_amd as fem
    dev = torch.device("cuda:0")
    res = {}

    def keep(key, t):
        res[key] = t.detach().cpu().numpy() if hasattr(t, "detach") else np.asarray(t)

    meshes = []
    for name, nodes, elems, a, b in _meshes():
        tn = torch.tensor(nodes, device=dev)
        te = torch.tensor(elems, device=dev)
        ta = torch.tensor(a, device=dev)
        tb = torch.tensor(b, device=dev)
        m = fem.Mesh(tn, te)
        for kind in ("ned", "rt"):
            K, M = fem.assemble(m, kind, tn, ta, tb)
            m.status()
            rowptr, colind = m.pattern(kind)
            keep(f"{name}_{kind}_K", K)
            keep(f"{name}_{kind}_M", M)
            keep(f"{name}_{kind}_rowptr", rowptr)
            keep(f"{name}_{kind}_colind", colind)
            rng = np.random.default_rng(5)
            u = torch.tensor(rng.normal(size=rowptr.numel() - 1), device=dev)
            rows = torch.repeat_interleave(torch.arange(rowptr.numel() - 1, device=dev), torch.diff(rowptr))
            w = u[rows] * u[colind.long()]
            gn, ga, gb = fem.assemble_backward(m, kind, tn, ta, tb, w, 0.5 * w)
            m.status()
            for k, v in (("gn", gn), ("ga", ga), ("gb", gb)):
                keep(f"{name}_{kind}_sep_{k}", v)
            gn, ga, gb = fem.assemble_backward(m, kind, tn, ta, tb, w, w)
            m.status()
            for k, v in (("gn", gn), ("ga", ga), ("gb", gb)):
                keep(f"{name}_{kind}_same_{k}", v)
            gn, ga, gb = fem.assemble_backward_quadratic(m, kind, tn, ta, tb, u)
            m.status()
            for k, v in (("gn", gn), ("ga", ga), ("gb", gb)):
                keep(f"{name}_{kind}_quad_{k}", v)
            _, _, L = fem.assemble_quadratic(m, kind, tn, ta, tb, u)
            m.status()
            keep(f"{name}_{kind}_L", L)
        meshes.append((name, m, tn, ta, tb))

    # batch: every tiling on the same meshes and kinds
    ms = [m for _, m, _, _, _ in meshes for _ in (0, 1)]
    kinds = ["ned", "rt"] * len(meshes)
    nodes = [tn for _, _, tn, _, _ in meshes for _ in (0, 1)]
    aa = [ta for _, _, _, ta, _ in meshes for _ in (0, 1)]
    bb = [tb for _, _, _, _, tb in meshes for _ in (0, 1)]
    Ks = [torch.empty(m.pattern_info(k)[1], dtype=torch.float64, device=dev) for m, k in zip(ms, kinds)]
    Ms = [torch.empty_like(K) for K in Ks]
    B = fem.Batch(ms, kinds)
    B.bind(nodes, aa, bb, Ks, Ms)
    for rows, threads, sched in ((0, 256, 1), (0, 128, 1), (64, 256, 1), (256, 256, 1), (0, 256, 4)):
        for K in Ks + Ms:
            K.fill_(float("nan"))
        B.set_config(rows, sched, threads)
        B.assemble()
        torch.cuda.synchronize()
        for m in ms:
            m.status()
        for i, (K, M) in enumerate(zip(Ks, Ms)):
            keep(f"batch{rows}_{threads}_{sched}_{i}_K", K)
            keep(f"batch{rows}_{threads}_{sched}_{i}_M", M)

    # Section 3.1 / 4.2: integration, load, error and CG on the eddy example
    from paper_1409_4618_amd.eddy import eddy_current
    n2, e2 = mg.unit_square(16)
    tn = torch.tensor(n2, device=dev)
    m = fem.Mesh(tn, torch.tensor(e2, device=dev))
    out = eddy_current(m, tn)
    m.status()
    keep("eddy_v", out["v"])
    keep("eddy_f", out["f"])
    keep("eddy_error", np.array([out["error"]]))
    per, tot = fem.norm_L2(m, tn, fem.FEM_FN_EDDY_E, per_elem=True)
    m.status()
    keep("norm_per", per)
    keep("norm_tot", tot)

    # Section 4.1: P1 system and the majorant pieces, 2D and 3D
    from paper_1409_4618_amd.majorant import minimise
    for name, (nd, el) in (("maj2", mg.unit_square(8)), ("maj3", mg.kuhn_box(4))):
        tn = torch.tensor(nd, device=dev)
        m = fem.Mesh(tn, torch.tensor(el, device=dev))
        r = minimise(m, tn)
        m.status()
        keep(f"{name}_M", np.array([it["majorant"] for it in r["iterations"]]))
        keep(f"{name}_beta", np.array([it["beta"] for it in r["iterations"]]))
        keep(f"{name}_err", np.array([r["error"]]))
    np.savez(os.path.join(out_dir, "results.npz"), **res)
    return res


if __name__ == "__main__":
    sys.path.insert(0, sys.argv[1])
    run(sys.argv[2])
    print("checked workload done", flush=True)
