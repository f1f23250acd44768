"""Batched launch: bitwise equal to single-mesh launches for every tile size
and schedule (the persistent kernel over every kind with schedules 0-2, one
launch per element kind with schedules 3-4), HIP-graph replays equal to
direct launches, and the autotuner's choice recorded in / read back from its
cache file."""
import json
import os

import numpy as np
import pytest

import meshgen as mg
import oracle
from gpu_util import TOL, dev_tensors, oracle_csr_many, rel_fro, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch_setup():
    import torch
    import paper_1409_4618_amd as fem
    probs = mg.batch_problems(seed=4, count=24, scale=0.02)
    say(f"[gpu] batch of {len(probs)} meshes, {sum(p.T for p in probs)} elements")
    meshes, kinds, nodes, a, b, Ks, Ms, refs = [], [], [], [], [], [], [], []
    for p in probs:
        tn, te, ta, tb = dev_tensors(p.nodes, p.elems, p.a, p.b)
        m = fem.Mesh(tn, te)
        K, M = fem.assemble(m, p.kind, tn, ta, tb)
        meshes.append(m)
        kinds.append(p.kind)
        nodes.append(tn)
        a.append(ta)
        b.append(tb)
        Ks.append(torch.full_like(K, float("nan")))
        Ms.append(torch.full_like(M, float("nan")))
        refs.append((K.clone(), M.clone()))
    torch.cuda.synchronize()
    return probs, meshes, kinds, nodes, a, b, Ks, Ms, refs


def test_single_meshes_match_oracle(batch_setup):
    probs, meshes, kinds, nodes, a, b, Ks, Ms, refs = batch_setup
    for i in (0, 1, len(probs) - 2, len(probs) - 1):
        p = probs[i]
        csr, _ = oracle.assemble(p.nodes, p.elems, p.kind, a=p.a, b=p.b)
        K, M = refs[i]
        assert rel_fro(K.cpu().numpy(), csr.Kv) <= TOL
        assert rel_fro(M.cpu().numpy(), csr.Mv) <= TOL


@pytest.mark.parametrize("rows,threads", [(0, 256), (0, 128), (64, 256), (128, 256), (256, 256)])
@pytest.mark.parametrize("schedule", [0, 1, 2, 3, 4])
def test_batch_equals_single_launches(batch_setup, rows, threads, schedule):
    import torch
    import paper_1409_4618_amd as fem
    probs, meshes, kinds, nodes, a, b, Ks, Ms, refs = batch_setup
    say(f"[gpu] batch rows={rows} threads={threads} schedule={schedule}")
    B = fem.Batch(meshes, kinds)
    for K, M in zip(Ks, Ms):
        K.fill_(float("nan"))
        M.fill_(float("nan"))
    B.bind(nodes, a, b, Ks, Ms)
    if rows != 0 and schedule > 2:
        # the per-kind launches exist for element-major tiles only
        with pytest.raises(fem.FemError):
            B.set_config(rows, schedule, threads)
        return
    B.set_config(rows, schedule, threads)
    B.assemble()
    B.assemble()  # the device work counter resets itself between launches
    torch.cuda.synchronize()
    for (K, M), (Kr, Mr) in zip(zip(Ks, Ms), refs):
        assert torch.equal(K, Kr) and torch.equal(M, Mr)
    cfg = B.config()
    assert cfg["rows_per_tile"] == rows and cfg["schedule"] == schedule and cfg["grid"] >= 1
    assert cfg["threads"] == threads
    if rows == 64 and schedule == 0:
        # workgroup sizes that do not go with the tiling are refused on the host
        for bad in ((64, 0, 128), (0, 0, 64), (0, 0, 0), (128, 1, 512)):
            with pytest.raises(fem.FemError):
                B.set_config(*bad)
        assert B.config()["rows_per_tile"] == 64


@pytest.mark.parametrize("rows,threads,schedule", [(0, 256, 1), (0, 256, 4), (0, 128, 3), (128, 256, 1)])
def test_graph_replay_equals_direct(batch_setup, rows, threads, schedule):
    import torch
    import paper_1409_4618_amd as fem
    probs, meshes, kinds, nodes, a, b, Ks, Ms, refs = batch_setup
    say(f"[gpu] batch graph replays, rows={rows} threads={threads} schedule={schedule}")
    B = fem.Batch(meshes, kinds)
    B.bind(nodes, a, b, Ks, Ms)
    B.set_config(rows, schedule, threads)
    for rep in range(3):
        for K, M in zip(Ks, Ms):
            K.zero_()
            M.zero_()
        B.graph_launch()
        torch.cuda.synchronize()
        for (K, M), (Kr, Mr) in zip(zip(Ks, Ms), refs):
            assert torch.equal(K, Kr) and torch.equal(M, Mr), rep
        # eager work between replays
        B.assemble()
        torch.cuda.synchronize()


def test_autotuner_and_cache(batch_setup, tmp_path):
    import torch
    import paper_1409_4618_amd as fem
    probs, meshes, kinds, nodes, a, b, Ks, Ms, refs = batch_setup
    say("[gpu] batch autotuner")
    cache = str(tmp_path / "fem_tune.jsonl")
    B = fem.Batch(meshes, kinds)
    B.bind(nodes, a, b, Ks, Ms)
    B.tune(cache)
    cfg = B.config()
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1
    rec = json.loads(lines[0])
    assert rec["rows_per_tile"] == cfg["rows_per_tile"] and rec["schedule"] == cfg["schedule"]
    assert rec["threads"] == cfg["threads"] and cfg["threads"] in (128, 256)
    # a second batch with the same signature reads the cache instead of timing
    B2 = fem.Batch(meshes, kinds)
    B2.bind(nodes, a, b, Ks, Ms)
    B2.set_config(64 if cfg["rows_per_tile"] != 64 else 128, 0)
    B2.tune(cache)
    assert B2.config()["rows_per_tile"] == cfg["rows_per_tile"]
    assert B2.config()["threads"] == cfg["threads"] and B2.config()["schedule"] == cfg["schedule"]
    assert len(open(cache).read().strip().splitlines()) == 1
    B2.assemble()
    torch.cuda.synchronize()
    for (K, M), (Kr, Mr) in zip(zip(Ks, Ms), refs):
        assert torch.equal(K, Kr) and torch.equal(M, Mr)


def test_full_size_batch_as_benchmarked():
    """The batched workload at its full size (256 meshes, 16.8 M elements) in the
    configuration the benchmark times (autotuned, graph replay): bitwise equal to
    single-mesh launches for every mesh, and every mesh equal to the oracle's
    full assembly (pattern bit-exact, values within relative Frobenius 1e-12)."""
    import torch
    import paper_1409_4618_amd as fem
    probs = mg.batch_problems(seed=4, count=256, scale=1.0)
    say(f"[gpu] full-size batch: {len(probs)} meshes, {sum(p.T for p in probs)} elements")
    meshes, kinds, nodes, a, b, Ks, Ms, refs = [], [], [], [], [], [], [], []
    for p in probs:
        tn, te, ta, tb = dev_tensors(p.nodes, p.elems, p.a, p.b)
        m = fem.Mesh(tn, te)
        K, M = fem.assemble(m, p.kind, tn, ta, tb)
        meshes.append(m)
        kinds.append(p.kind)
        nodes.append(tn)
        a.append(ta)
        b.append(tb)
        refs.append((K, M))
        Ks.append(torch.full_like(K, float("nan")))
        Ms.append(torch.full_like(M, float("nan")))
    B = fem.Batch(meshes, kinds)
    B.bind(nodes, a, b, Ks, Ms)
    B.tune(None)
    say(f"    tuned: {B.config()}")
    for _ in range(2):
        B.graph_launch()
    torch.cuda.synchronize()
    for i, ((K, M), (Kr, Mr)) in enumerate(zip(zip(Ks, Ms), refs)):
        assert torch.equal(K, Kr) and torch.equal(M, Mr), i
    for m in meshes:
        m.status()
    # every mesh against the oracle's full assembly (CPU worker processes)
    say("    oracle: full assembly of every mesh")
    worst = 0.0
    for i, (rp, ci, Kv, Mv) in enumerate(oracle_csr_many(probs)):
        rowptr, colind = meshes[i].pattern(kinds[i])
        assert np.array_equal(rowptr.cpu().numpy(), rp) and np.array_equal(colind.cpu().numpy(), ci), i
        K, M = refs[i]
        eK, eM = rel_fro(K.cpu().numpy(), Kv), rel_fro(M.cpu().numpy(), Mv)
        worst = max(worst, eK, eM)
        assert eK <= TOL and eM <= TOL, (i, eK, eM)
    say(f"    all {len(probs)} meshes: worst rel Frobenius error {worst:.2e}")


def test_launches_are_ordered_with_the_callers_stream(batch_setup):
    """The first graph launch (which runs one plain launch before capturing)
    and a rebind both wait for work already queued by the caller: a read of K
    queued behind a spin on the caller's stream still sees the old values, and
    a launch queued before a rebind still writes the buffers it was bound to."""
    import torch
    import paper_1409_4618_amd as fem
    probs, meshes, kinds, nodes, a, b, Ks, Ms, refs = batch_setup
    say("[gpu] batch launches ordered with the caller's stream")
    s = torch.cuda.Stream()
    B = fem.Batch(meshes, kinds)
    B.bind(nodes, a, b, Ks, Ms)
    B.set_config(0, 1)
    for K, M in zip(Ks, Ms):
        K.fill_(-1.0)
        M.fill_(-1.0)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        torch.cuda._sleep(20_000_000)
        seen = Ks[-1].clone()
        B.graph_launch()
    torch.cuda.synchronize()
    assert bool((seen == -1.0).all())
    for (K, M), (Kr, Mr) in zip(zip(Ks, Ms), refs):
        assert torch.equal(K, Kr) and torch.equal(M, Mr)
    # a launch queued behind a spin, then a rebind to fresh outputs
    Ks2 = [torch.full_like(K, -2.0) for K in Ks]
    Ms2 = [torch.full_like(M, -2.0) for M in Ms]
    for K, M in zip(Ks, Ms):
        K.fill_(-1.0)
        M.fill_(-1.0)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        torch.cuda._sleep(20_000_000)
        B.assemble()
    B.bind(nodes, a, b, Ks2, Ms2)
    torch.cuda.synchronize()
    for (K, M), (Kr, Mr) in zip(zip(Ks, Ms), refs):
        assert torch.equal(K, Kr) and torch.equal(M, Mr)
    assert all(bool((K == -2.0).all()) for K in Ks2)
    B.assemble()
    torch.cuda.synchronize()
    for (K, M), (Kr, Mr) in zip(zip(Ks2, Ms2), refs):
        assert torch.equal(K, Kr) and torch.equal(M, Mr)


def test_binding_rejects_bad_buffers(batch_setup):
    """Buffers of the wrong size, type or device are refused by the binding
    before any kernel could write past them."""
    import torch
    import paper_1409_4618_amd as fem
    probs, meshes, kinds, nodes, a, b, Ks, Ms, refs = batch_setup
    say("[gpu] binding argument checks")
    B = fem.Batch(meshes[:2], kinds[:2])
    short = Ks[1][:-1]
    with pytest.raises(ValueError):
        B.bind(nodes[:2], a[:2], b[:2], [Ks[0], short], Ms[:2])
    with pytest.raises(ValueError):
        B.bind(nodes[:2], a[:2], b[:2], Ks[:1], Ms[:2])
    with pytest.raises(ValueError):
        B.bind(nodes[:2], [a[0], a[1].float()], b[:2], Ks[:2], Ms[:2])
    with pytest.raises(ValueError):
        fem.assemble_into(meshes[0], kinds[0], nodes[0], a[0], b[0], Ks[0], Ms[0][:-1])
    with pytest.raises(ValueError):
        fem.assemble_into(meshes[0], kinds[0], nodes[0], a[0][:-1], b[0], Ks[0], Ms[0])
    with pytest.raises(ValueError):
        fem.assemble_into(meshes[0], kinds[0], nodes[0].cpu(), a[0], b[0], Ks[0], Ms[0])
    torch.cuda.synchronize()
