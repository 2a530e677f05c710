"""The graph-growing start (jet_bfs_start, JET_F_BFS_START) against the CPU
oracle: the start itself element by element on graphs with one or many
components, isolated vertices, vertex weights and ragged sizes; the full
multilevel partition from it (trace of every level and the final
partition); and serving jobs with the flag against the same job alone."""
import numpy as np
import pytest

from paper_2304_13194_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


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


START_CASES = [
    ("single_vertex", I.csr_from_edges(1, np.zeros(0, np.int64), np.zeros(0, np.int64)), False),
    ("path9", I.csr_from_edges(9, np.arange(8), np.arange(1, 9)), True),
    ("grid37x29", I.grid2d(37, 29), True),
    ("stencil12", I.stencil27(12, 12, 12), True),
    ("er300_weighted_components", I.small_random_graph(300, 0.008, 4, wmax=5, vwmax=7), False),
    ("rmat12_isolated", I.rmat(12, 8, 3), False),
    ("star2000", I.csr_from_edges(2001, np.full(2000, 1000, np.int64),
                                  np.concatenate([np.arange(0, 1000), np.arange(1001, 2001)])), True),
    ("rgg5000", I.rgg(5000, 2), True),
]


@pytest.mark.parametrize("case", START_CASES, ids=[c[0] for c in START_CASES])
def test_bfs_start_matches_oracle(J, O, case):
    name, g, unit = case
    dg = J.to_device(g, unit_vwgt=unit, unit_adjwgt=unit)
    for k in (1, 3, 64, 1000):
        _say(f"bfs start {name} n={g.n} k={k}")
        part = J.bfs_start(dg, k).cpu().numpy()
        np.testing.assert_array_equal(part, O.bfs_part(g, k), err_msg=f"{name} k={k}")


def test_bfs_start_errors(J):
    import torch
    g = I.grid2d(6, 6)
    dg = J.to_device(g)
    with pytest.raises(J.JetError) as e:
        J.bfs_start(dg, 0)
    assert e.value.status == J.JET_EINVAL
    with pytest.raises(J.JetError) as e:
        J.bfs_start(dg, 16385)
    assert e.value.status == J.JET_ELIMIT
    bad = dg.adjncy.clone()
    bad[0] = g.n + 3
    with pytest.raises(J.JetError) as e:
        J.bfs_start(J.DeviceGraph(dg.xadj, bad, dg.vwgt, dg.adjwgt), 4)
    assert e.value.status == J.JET_EGRAPH
    torch.cuda.synchronize()


PART_CASES = [
    ("grid40_k4", I.grid2d(40, 40), 4, 3),
    ("stencil16_k8", I.stencil27(16, 16, 16), 8, 5),
    ("rmat13_k16", I.rmat(13, 8, 4), 16, 6),
    ("rgg20000_k32", I.rgg(20000, 3), 32, 7),
    ("er200_k2", I.small_random_graph(200, 0.05, 9, wmax=5, vwmax=3), 2, 8),
]


@pytest.mark.parametrize("case", PART_CASES, ids=[c[0] for c in PART_CASES])
def test_partition_from_bfs_start_matches_oracle(J, O, case):
    name, g, k, seed = case
    _say(f"partition from the graph-growing start {name} n={g.n} k={k}")
    exp = O.partition(g, k, seed=seed, flags=O.F_BFS_START)
    part, st, tr = J.partition(J.to_device(g), k, seed=seed, trace_cap=100000, flags=J.JET_F_BFS_START)
    assert st["levels"] == len(exp["level_sizes"])
    assert len(tr) == len(exp["trace"])
    for a, b in zip(tr, exp["trace"]):
        assert a == b, f"{name}: gpu {a} != oracle {b}"
    np.testing.assert_array_equal(part.cpu().numpy(), exp["part"])
    assert st["cut"] == exp["cut"] and bool(st["balanced"]) == exp["balanced"]


def test_server_jobs_with_bfs_start_equal_alone(J):
    import torch
    jobs = [(I.grid2d(64, 64), True, 8, 1), (I.rmat(12, 8, 5), False, 32, 2), (I.stencil27(10, 10, 10), True, 4, 3)]
    dgs = [J.to_device(g, unit_vwgt=u, unit_adjwgt=u) for g, u, _, _ in jobs]
    alone = [J.partition(dg, k, seed=s, flags=J.JET_F_BFS_START)[0].cpu().numpy()
             for dg, (_, _, k, s) in zip(dgs, jobs)]
    outs = [torch.full((dg.n,), -1, dtype=torch.int32, device="cuda") for dg in dgs]
    torch.cuda.synchronize()
    sv = J.Server(max_slots=4)
    try:
        tickets = [sv.submit(dg, o, k, seed=s, flags=J.JET_F_BFS_START)
                   for dg, o, (_, _, k, s) in zip(dgs, outs, jobs)]
        res = [sv.wait(t, 120000) for t in tickets]
    finally:
        sv.close()
    for i, (r, o, a) in enumerate(zip(res, outs, alone)):
        assert r["status"] == 0, i
        np.testing.assert_array_equal(o.cpu().numpy(), a, err_msg=f"job {i}")
