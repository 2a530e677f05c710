"""Parity at the benchmark's full sizes, through the calls bench.py times.

* 3-D 27-point stencil 128^3 (n = 2,097,152, 2m = 53,645,816), k = 64,
  lambda 3%, seed 2: the whole multilevel partition (jet_partition with the
  profiling flag and a trace, as timed) against the oracle's partition of the
  same graph: every per-iteration trace record of every level (kind, counts,
  cut, largest part weight, best cut, partition digest), the final partition
  element by element, cut and balance. The same call without the profiling
  flag, where every level replays its iteration pairs as HIP graphs, gives
  the same partition. The partition from the graph-growing start of the
  coarsest graph (JET_F_BFS_START) matches the oracle's the same way.
* The 512-RGG batch (sum n = 18.0M, sum 2m = 180M): one jet_refine_batch
  call as timed (autotuned work-queue tile and group width). Every graph
  equals jet_refine of that graph alone; sampled graphs match the oracle's
  refinement of each graph alone; for every graph the part ids lie in
  [0, k), and the cut and the largest part weight recomputed from the
  returned partition equal the reported ones.
* Serving: the first 40 jobs of the serving mix (grids up to 1024^2, R-MAT up
  to scale 20) submitted at once; every result equals jet_partition of the
  same job alone, and sampled jobs equal the oracle's partition.
"""
import multiprocessing as mp
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

from paper_2304_13194_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def J():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_13194_amd import jet
    jet.lib()
    return jet


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    oracle.lib()
    return oracle


def _pool():
    # input generation only (numpy); spawned workers never touch the GPU
    return ProcessPoolExecutor(max_workers=8, mp_context=mp.get_context("spawn"))


def _recount(g, part, k):
    """Cut and part weights of `part`, recomputed from the CSR graph."""
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.xadj))
    diff = part[src] != part[g.adjncy]
    cut = int(np.sum(g.adjwgt[diff].astype(np.int64))) // 2
    pw = np.bincount(part, weights=g.vwgt, minlength=k).astype(np.int64)
    return cut, pw


def test_stencil128_partition_matches_oracle(J, O):
    import torch
    t0 = time.perf_counter()
    g = I.stencil27(128, 128, 128)
    k, seed = 64, 2
    _say(f"stencil128: n={g.n} 2m={g.nnz} generated in {time.perf_counter() - t0:.1f} s")
    dg = J.to_device(g, unit_vwgt=True, unit_adjwgt=True)
    part, st, tr = J.partition(dg, k, seed=seed, flags=J.JET_F_PROFILE, trace_cap=1 << 16)
    part = part.cpu().numpy()
    part2, st2, _ = J.partition(dg, k, seed=seed)
    torch.cuda.synchronize()
    _say(f"gpu: cut={st['cut']} iters={st['iters']} levels={st['levels']}; oracle running")
    t0 = time.perf_counter()
    exp = O.partition(g, k, seed=seed, trace_cap=1 << 20)
    _say(f"oracle: cut={exp['cut']} in {time.perf_counter() - t0:.1f} s")
    assert st["levels"] == len(exp["level_sizes"])
    assert len(tr) == len(exp["trace"])
    for a, b in zip(tr, exp["trace"]):
        assert a == b, f"gpu {a} != oracle {b}"
    np.testing.assert_array_equal(part, exp["part"])
    assert st["cut"] == exp["cut"] and bool(st["balanced"]) == exp["balanced"]
    np.testing.assert_array_equal(part2.cpu().numpy(), part)
    assert st2["cut"] == st["cut"] and st2["iters"] == st["iters"]
    cut, pw = _recount(g, part, k)
    assert cut == st["cut"] and int(pw.max()) == st["max_part_weight"] and int(pw.sum()) == g.n


def test_stencil128_partition_from_bfs_start_matches_oracle(J, O):
    """The same partition started from the graph-growing partition of the
    coarsest graph (JET_F_BFS_START): every trace record and the result."""
    g = I.stencil27(128, 128, 128)
    k, seed = 64, 2
    dg = J.to_device(g, unit_vwgt=True, unit_adjwgt=True)
    part, st, tr = J.partition(dg, k, seed=seed, flags=J.JET_F_BFS_START, trace_cap=1 << 16)
    part = part.cpu().numpy()
    _say(f"gpu (graph-growing start): cut={st['cut']} iters={st['iters']}; oracle running")
    exp = O.partition(g, k, seed=seed, flags=O.F_BFS_START, trace_cap=1 << 20)
    assert len(tr) == len(exp["trace"])
    for a, b in zip(tr, exp["trace"]):
        assert a == b, f"gpu {a} != oracle {b}"
    np.testing.assert_array_equal(part, exp["part"])
    assert st["cut"] == exp["cut"] and bool(st["balanced"]) == exp["balanced"]


def test_rgg512_batch_full_size(J, O):
    import torch
    spec = I.rgg_batch_spec()
    t0 = time.perf_counter()
    with _pool() as ex:
        graphs = list(ex.map(I.rgg, [n for n, _, _ in spec], [s for _, _, s in spec], chunksize=8))
    _say(f"512 RGGs: sum n={sum(g.n for g in graphs)} sum 2m={sum(g.nnz for g in graphs)} "
         f"generated in {time.perf_counter() - t0:.1f} s")
    dgs = [J.to_device(g, unit_vwgt=True, unit_adjwgt=True) for g in graphs]
    p0 = [I.random_partition(g.n, k, s) for g, (n, k, s) in zip(graphs, spec)]
    parts = [torch.from_numpy(p.copy()).cuda() for p in p0]
    params = [dict(k=k, seed=s) for (n, k, s) in spec]
    stats, _ = J.refine_batch(dgs, parts, params)
    torch.cuda.synchronize()
    host = [p.cpu().numpy() for p in parts]
    for i, (g, (n, k, s), part, st) in enumerate(zip(graphs, spec, host, stats)):
        assert part.min() >= 0 and part.max() < k, i
        cut, pw = _recount(g, part, k)
        assert cut == st["cut"], f"graph {i}: recomputed cut {cut} != {st['cut']}"
        assert int(pw.max()) == st["max_part_weight"] and int(pw.sum()) == g.n, i
        assert bool(st["balanced"]) == (st["max_part_weight"] <= st["o"]), i
    # every graph equals its refinement alone (jet_refine, one launch sequence each)
    single = [torch.from_numpy(p.copy()).cuda() for p in p0]
    for dg, p, prm in zip(dgs, single, params):
        J.refine(dg, p, **prm)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(host, single)):
        np.testing.assert_array_equal(a, b.cpu().numpy(), err_msg=f"graph {i}: batch vs alone")
    _say(f"all {len(spec)} graphs equal their alone runs (tile {stats[0]['batch_tile']}, "
         f"groups of {stats[0]['batch_group']})")
    # sampled graphs against the oracle: seeded picks plus the largest graph
    u = I.stream(4242, np.arange(9, dtype=np.uint64))
    pick = sorted(set(I.uniform_below(u, len(spec)).tolist()) | {int(np.argmax([n for n, _, _ in spec]))})
    for i in pick:
        n, k, s = spec[i]
        exp = O.refine(graphs[i], p0[i], k, seed=s)
        _say(f"  graph {i}: n={n} k={k} iters gpu={stats[i]['iters']} oracle={exp.iters} cut={stats[i]['cut']}")
        assert stats[i]["iters"] == exp.iters, i
        np.testing.assert_array_equal(host[i], exp.part, err_msg=f"graph {i}")
        assert stats[i]["cut"] == exp.cut and stats[i]["max_part_weight"] == exp.maxw, i


def test_serving_mix_full_size(J, O):
    import torch
    jobs = I.serve_jobs(40)
    t0 = time.perf_counter()
    with _pool() as ex:
        pool = list(ex.map(I.serve_pool_graph, I.SERVE_POOL))
    _say(f"serving pool generated in {time.perf_counter() - t0:.1f} s")
    unit = [s[0] == "grid" for s in I.SERVE_POOL]
    dgs = [J.to_device(g, unit_vwgt=u, unit_adjwgt=u) for g, u in zip(pool, unit)]
    alone = []
    for gi, k, seed in jobs:
        part, st, _ = J.partition(dgs[gi], k, seed=seed)
        alone.append((part.cpu().numpy(), st))
    outs = [torch.full((dgs[gi].n,), -1, dtype=torch.int32, device="cuda") for gi, _, _ in jobs]
    torch.cuda.synchronize()
    sv = J.Server(hbm_budget_bytes=128 << 30, max_slots=64)
    try:
        tickets = [sv.submit(dgs[gi], o, k, seed=seed) for (gi, k, seed), o in zip(jobs, outs)]
        res = [sv.wait(t, 600000) for t in tickets]
        info = sv.info()
    finally:
        sv.close()
    _say(f"served {info['completed']} jobs in {info['steps']} steps")
    for j, ((gi, k, seed), o, r, (pa, sa)) in enumerate(zip(jobs, outs, res, alone)):
        assert r["status"] == 0, j
        np.testing.assert_array_equal(o.cpu().numpy(), pa, err_msg=f"job {j}")
        assert r["cut"] == sa["cut"] and r["iters"] == sa["iters"], j
    # the oracle on the largest grid job and the largest R-MAT job of the mix
    sizes = [pool[gi].nnz for gi, _, _ in jobs]
    grid_jobs = [j for j, (gi, _, _) in enumerate(jobs) if unit[gi]]
    rmat_jobs = [j for j, (gi, _, _) in enumerate(jobs) if not unit[gi]]
    for j in (max(grid_jobs, key=lambda x: sizes[x]), max(rmat_jobs, key=lambda x: sizes[x])):
        gi, k, seed = jobs[j]
        t0 = time.perf_counter()
        exp = O.partition(pool[gi], k, seed=seed)
        _say(f"  job {j}: {I.SERVE_POOL[gi]} k={k} oracle in {time.perf_counter() - t0:.1f} s")
        np.testing.assert_array_equal(outs[j].cpu().numpy(), exp["part"], err_msg=f"job {j}")
        assert res[j]["cut"] == exp["cut"], j
