"""Helpers shared by the GPU tests (not a test module)."""
import sys

import numpy as np

TOL = 1e-12  # relative Frobenius error bound for K and M values


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def dev_tensors(nodes, elems, a=None, b=None):
    import torch
    d = torch.device("cuda:0")
    tn = torch.tensor(np.ascontiguousarray(nodes), dtype=torch.float64, device=d)
    te = torch.tensor(np.ascontiguousarray(elems), dtype=torch.int32, device=d)
    ta = None if a is None else torch.tensor(a, dtype=torch.float64, device=d)
    tb = None if b is None else torch.tensor(b, dtype=torch.float64, device=d)
    return tn, te, ta, tb


def rel_fro(got, ref):
    ref = np.asarray(ref)
    den = np.linalg.norm(ref)
    return np.linalg.norm(np.asarray(got) - ref) / (den if den > 0 else 1.0)


def relabel(nodes, elems, seed):
    """Random node relabelling and random local vertex order (mixed orientations)."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(nodes.shape[0])
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    e2 = inv[elems]
    idx = np.argsort(rng.random(e2.shape), axis=1)
    e2 = np.take_along_axis(e2, idx, axis=1)
    return nodes[perm], e2.astype(np.int32)


def csr_rows_of(rowptr, colind, vals, r):
    s, e = int(rowptr[r]), int(rowptr[r + 1])
    return colind[s:e], vals[s:e]


def _oracle_csr(args):
    """Worker: the oracle's full assembly of one mesh (CPU only)."""
    import oracle
    nodes, elems, kind, a, b = args
    csr, _ = oracle.assemble(nodes, elems, kind, a=a, b=b)
    return csr.rowptr, csr.colind, csr.Kv, csr.Mv


def oracle_csr_many(problems, workers=12):
    """The oracle's full assembly of many meshes, in spawned CPU worker
    processes (they import numpy and the oracle only, never the GPU)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    jobs = [(p.nodes, p.elems, p.kind, p.a, p.b) for p in problems]
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_oracle_csr, jobs, chunksize=1))
