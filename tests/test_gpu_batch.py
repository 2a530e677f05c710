"""GPU parity of batched refinement (jet_refine_batch) against the CPU oracle.

Every graph of a batch must come out exactly as the oracle refines it alone:
P_best, cut, part weights bound, iteration count and every per-iteration
trace record (partition digest included). The batches mix sizes, k, levels,
seeds, weighted and unit graphs, every degree class and the trivial cases
(k = 1, n = 0) the call answers directly.
"""
import sys

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


def star(nleaves):
    return I.csr_from_edges(nleaves + 1, np.zeros(nleaves, np.int64), np.arange(1, nleaves + 1))


def _skewed(n, k, seed):
    x = I.stream(seed, np.arange(n, dtype=np.uint64))
    y = I.stream(seed + 1, np.arange(n, dtype=np.uint64))
    return np.where(I.uniform_below(x, 3) == 0, I.uniform_below(y, k), I.uniform_below(y, max(1, k // 3)))\
        .astype(np.int32)


def mixed_jobs():
    """(name, graph, unit weights?, k, level, seed, P_0)."""
    spec = [
        ("grid40_k4", I.grid2d(40, 40), True, 4, 0, 3),
        ("rmat12_k32_w", I.rmat(12, 8, 5), False, 32, 0, 7),
        ("stencil10_k8_l1", I.stencil27(10, 10, 10), True, 8, 1, 1),
        ("er0_k2", I.small_random_graph(41, 0.15, 700, wmax=3, vwmax=2), False, 2, 0, 5),
        ("star2000_k3", star(2000), True, 3, 0, 9),
        ("rmat13_k64_hubs", I.rmat(13, 16, 6), False, 64, 2, 2),
        ("rgg2500_k16", I.rgg(2500, 9), True, 16, 0, 4),
        ("er1_k5", I.small_random_graph(63, 0.2, 701, wmax=5, vwmax=3), False, 5, 1, 8),
        ("rmat11_k200", I.rmat(11, 8, 9), False, 200, 0, 6),
    ]
    jobs = []
    for i, (name, g, unit, k, level, seed) in enumerate(spec):
        P0 = I.random_partition(g.n, k, 500 + i) if i % 2 == 0 else _skewed(g.n, k, 600 + i)
        jobs.append((name, g, unit, k, level, seed, P0))
    return jobs


def _device(J, g, unit):
    return J.to_device(g, unit_vwgt=unit, unit_adjwgt=unit)


def _run_batch(J, jobs, trace_cap=4096):
    import torch
    graphs = [_device(J, g, unit) for _, g, unit, _, _, _, _ in jobs]
    parts = [torch.from_numpy(P0.copy()).cuda() for *_, P0 in jobs]
    params = [dict(k=k, level=level, seed=seed) for _, _, _, k, level, seed, _ in jobs]
    stats, traces = J.refine_batch(graphs, parts, params, trace_cap=trace_cap)
    return [p.cpu().numpy() for p in parts], stats, traces


def _check_against_oracle(O, jobs, parts, stats, traces):
    for (name, g, unit, k, level, seed, P0), part, st, tr in zip(jobs, parts, stats, traces):
        exp = O.refine(g, P0, k, level=level, seed=seed)
        _say(f"  {name}: n={g.n} k={k} iters gpu={st['iters']} oracle={exp.iters} cut={st['cut']}")
        assert st["iters"] == exp.iters, name
        assert len(tr) == len(exp.trace), name
        for a, b in zip(tr, exp.trace):
            assert a == b, f"{name}: gpu {a} != oracle {b}"
        np.testing.assert_array_equal(part, exp.part, err_msg=name)
        assert st["cut"] == exp.cut and st["max_part_weight"] == exp.maxw, name
        assert bool(st["balanced"]) == exp.balanced, name


def test_batch_matches_oracle_mixed(J, O):
    jobs = mixed_jobs()
    _say(f"batch of {len(jobs)} mixed graphs")
    parts, stats, traces = _run_batch(J, jobs)
    _check_against_oracle(O, jobs, parts, stats, traces)


def test_batch_equals_alone(J):
    """Each graph's result is the same alone (jet_refine) and in the batch."""
    import torch
    jobs = mixed_jobs()
    parts, stats, traces = _run_batch(J, jobs)
    for (name, g, unit, k, level, seed, P0), part, st, tr in zip(jobs, parts, stats, traces):
        p = torch.from_numpy(P0.copy()).cuda()
        s1, t1, _ = J.refine(_device(J, g, unit), p, k, trace_cap=4096, level=level, seed=seed)
        np.testing.assert_array_equal(p.cpu().numpy(), part, err_msg=name)
        assert t1 == tr and s1["cut"] == st["cut"] and s1["iters"] == st["iters"], name


def test_batch_trivial_and_order(J, O):
    """k = 1 and n = 0 graphs inside a batch, a high-k graph next to a tiny one,
    and the same graph twice with different seeds."""
    import torch
    g = I.rmat(11, 8, 3)
    tiny = I.small_random_graph(12, 0.3, 9, wmax=2, vwmax=2)
    empty = I.csr_from_edges(0, np.zeros(0, np.int64), np.zeros(0, np.int64))
    jobs = [
        ("rmat11_k1", g, False, 1, 0, 0, np.zeros(g.n, np.int32)),
        ("rmat11_k600", g, False, 600, 0, 1, I.random_partition(g.n, 600, 31)),
        ("tiny_k3", tiny, False, 3, 0, 2, I.random_partition(tiny.n, 3, 32)),
        ("empty_k4", empty, True, 4, 0, 0, np.zeros(0, np.int32)),
        ("rmat11_k8_s1", g, False, 8, 0, 1, I.random_partition(g.n, 8, 33)),
        ("rmat11_k8_s2", g, False, 8, 0, 2, I.random_partition(g.n, 8, 33)),
    ]
    parts, stats, traces = _run_batch(J, jobs)
    assert (parts[0] == 0).all() and stats[0]["iters"] == 0
    assert parts[3].shape == (0,)
    live = [i for i in range(len(jobs)) if i not in (0, 3)]
    _check_against_oracle(O, [jobs[i] for i in live], [parts[i] for i in live], [stats[i] for i in live],
                          [traces[i] for i in live])


def rgg_batch(count, nmin, nmax, seed):
    """RGG batch shaped like the paper's batched workload (n log-uniform,
    mean degree about 10, k from {2, ..., 128}, unit weights)."""
    u = I.stream(seed, np.arange(2 * count, dtype=np.uint64))
    lo, hi = np.log(nmin), np.log(nmax)
    jobs = []
    for i in range(count):
        frac = float(u[i] >> np.uint64(11)) / float(1 << 53)
        n = int(np.exp(lo + (hi - lo) * frac))
        k = [2, 4, 8, 16, 32, 64, 128][int(I.uniform_below(u[count + i:count + i + 1], 7)[0])]
        g = I.rgg(n, seed * 1000 + i)
        jobs.append((f"rgg{i}_n{n}_k{k}", g, True, k, 0, seed + i, I.random_partition(n, k, seed * 7 + i)))
    return jobs


def test_batch_rgg_workload(J, O):
    jobs = rgg_batch(24, 1000, 20000, 5)
    _say(f"rgg batch: {len(jobs)} graphs, {sum(j[1].n for j in jobs)} vertices")
    parts, stats, traces = _run_batch(J, jobs, trace_cap=8192)
    _check_against_oracle(O, jobs, parts, stats, traces)


def test_batch_errors(J):
    import torch
    g = I.grid2d(10, 10)
    dg = _device(J, g, True)
    good = torch.from_numpy(I.random_partition(g.n, 4, 1)).cuda()
    bad = good.clone()
    bad[17] = 4  # part id out of range for k = 4
    with pytest.raises(J.JetError) as e:
        J.refine_batch([dg, dg], [good.clone(), bad], [dict(k=4), dict(k=4)])
    assert e.value.status == J.JET_EPART
    # a neighbour id outside its own graph (it would be a vertex of the next graph in the union)
    adj = dg.adjncy.clone()
    adj[5] = g.n
    broken = J.DeviceGraph(dg.xadj, adj, None, None)
    with pytest.raises(J.JetError) as e:
        J.refine_batch([broken, dg], [good.clone(), good.clone()], [dict(k=4), dict(k=4)])
    assert e.value.status == J.JET_EGRAPH
    with pytest.raises(J.JetError) as e:
        J.refine_batch([dg], [good.clone()], [dict(k=0)])
    assert e.value.status == J.JET_EINVAL
    stats, traces = J.refine_batch([], [], [])
    assert stats == [] and traces is None


def _alone(J, jobs):
    import torch
    out = []
    for name, g, unit, k, level, seed, P0 in jobs:
        p = torch.from_numpy(P0.copy()).cuda()
        st, tr, _ = J.refine(_device(J, g, unit), p, k, trace_cap=4096, level=level, seed=seed)
        out.append((p.cpu().numpy(), st, tr))
    return out


@pytest.mark.parametrize("tile,group", [(0, 8), (1, 4), (64, 4)], ids=["static_g8", "tile1_g4", "tile64_g4"])
def test_batch_work_queue_choices_identical(J, monkeypatch, tile, group):
    """Forced autotuner choices (static walks, or work-queue tiles of 1 or 64
    visits per wave taken from per-XCD sub-queues; 4- or 8-lane groups for
    small rows) and a reversed batch order all give every graph its result
    alone, trace included."""
    jobs = [j for j in rgg_batch(30, 1000, 30000, 6) if j[3] <= 64] + mixed_jobs()[:4]
    jobs = [j for j in jobs if j[3] <= 64]
    alone = _alone(J, jobs)
    monkeypatch.setenv("JET_BATCH_TILE", str(tile))
    monkeypatch.setenv("JET_BATCH_GROUP", str(group))
    for order in (list(range(len(jobs))), list(reversed(range(len(jobs))))):
        batch = [jobs[i] for i in order]
        parts, stats, traces = _run_batch(J, batch)
        assert all(s["batch_tile"] == tile and s["batch_group"] == group for s in stats)
        for j, i in enumerate(order):
            p, st, tr = alone[i]
            np.testing.assert_array_equal(parts[j], p, err_msg=jobs[i][0])
            assert traces[j] == tr and stats[j]["cut"] == st["cut"], jobs[i][0]


def test_batch_autotuned_equals_alone(J):
    """A batch large enough for the autotuner (over 2^20 CSR entries): its
    measured choice is recorded, and every graph equals its alone run."""
    jobs = rgg_batch(40, 10000, 100000, 7)
    assert sum(j[1].nnz for j in jobs) >= 1 << 20
    alone = _alone(J, jobs)
    parts, stats, traces = _run_batch(J, jobs)
    _say(f"autotuned: tile {stats[0]['batch_tile']} visits, groups of {stats[0]['batch_group']} lanes")
    assert stats[0]["batch_tile"] in (0, 16, 64) and stats[0]["batch_group"] in (4, 8)
    for (name, *_), part, st, tr, (p, s1, t1) in zip(jobs, parts, stats, traces, alone):
        np.testing.assert_array_equal(part, p, err_msg=name)
        assert tr == t1 and st["cut"] == s1["cut"], name
