"""The serving loop (jet_server_*): results alone and in the mix.

A job served next to others (continuous batching at level granularity,
admission by slots and HBM footprint, jobs arriving while others run) must
come out bit-identical to the same job partitioned alone by jet_partition,
and small jobs are also checked against the CPU oracle's multilevel
partition.
"""
import sys
import time

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


def job_mix():
    """(name, host graph, unit weights?, k, seed)."""
    return [
        ("grid96_k16", I.grid2d(96, 96), True, 16, 1),
        ("rmat13_k64", I.rmat(13, 8, 21), False, 64, 2),
        ("grid40_k4", I.grid2d(40, 40), True, 4, 3),
        ("rmat12_k200", I.rmat(12, 16, 22), False, 200, 4),
        ("stencil16_k8", I.stencil27(16, 16, 16), True, 8, 5),
        ("grid64_k2", I.grid2d(64, 64), True, 2, 6),
        ("rmat14_k32", I.rmat(14, 8, 23), False, 32, 7),
        ("grid128_k256", I.grid2d(128, 128), True, 256, 8),
    ]


def _alone(J, jobs, dgs):
    out = []
    for (name, g, unit, k, seed), dg in zip(jobs, dgs):
        part, st, _ = J.partition(dg, k, seed=seed)
        out.append((part.cpu().numpy(), st))
    return out


def _serve(J, jobs, dgs, slots, budget=0, stagger_s=0.0):
    import torch
    sv = J.Server(hbm_budget_bytes=budget, max_slots=slots)
    try:
        parts = [torch.full((dg.n,), -1, dtype=torch.int32, device="cuda") for dg in dgs]
        torch.cuda.synchronize()
        tickets = []
        seen = dict(max_queued=0, max_in_use=0)
        for i, ((name, g, unit, k, seed), dg) in enumerate(zip(jobs, dgs)):
            tickets.append(sv.submit(dg, parts[i], k, seed=seed))
            inf = sv.info()
            seen["max_queued"] = max(seen["max_queued"], inf["queued"])
            seen["max_in_use"] = max(seen["max_in_use"], inf["hbm_in_use"])
            if stagger_s and i % 3 == 2:
                time.sleep(stagger_s)
        res = []
        for t in tickets:
            res.append(sv.wait(t, 120000))
            inf = sv.info()
            seen["max_in_use"] = max(seen["max_in_use"], inf["hbm_in_use"])
        info = sv.info()
        info.update(seen)
    finally:
        sv.close()
    return [p.cpu().numpy() for p in parts], res, info


def test_server_mix_equals_alone(J):
    jobs = job_mix()
    dgs = [J.to_device(g, unit_vwgt=unit, unit_adjwgt=unit) for _, g, unit, _, _ in jobs]
    alone = _alone(J, jobs, dgs)
    for slots, stagger in ((4, 0.0), (8, 0.02), (1, 0.0)):
        parts, res, info = _serve(J, jobs, dgs, slots, stagger_s=stagger)
        _say(f"slots={slots} stagger={stagger}: steps={info['steps']} jobs/step="
             f"{info['step_jobs'] / max(info['steps'], 1):.2f}")
        assert info["completed"] == len(jobs)
        for (name, *_), p, r, (pa, sa) in zip(jobs, parts, res, alone):
            assert r is not None and r["status"] == 0, name
            np.testing.assert_array_equal(p, pa, err_msg=f"{name} slots={slots}")
            assert r["cut"] == sa["cut"] and r["iters"] == sa["iters"] and r["levels"] == sa["levels"], name
            assert r["t_submit_ms"] <= r["t_admit_ms"] <= r["t_done_ms"], name
        if slots > 1:
            assert info["step_jobs"] > info["steps"], "jobs never shared a step"


def test_server_budget_admission(J):
    jobs = job_mix()[:5]
    dgs = [J.to_device(g, unit_vwgt=unit, unit_adjwgt=unit) for _, g, unit, _, _ in jobs]
    alone = _alone(J, jobs, dgs)
    # a budget that fits the largest job but never two of the large ones together
    fp = [3 * (8 * (dg.n + 1) + 4 * dg.nnz * (2 if dg.adjwgt is not None else 1) +
               (4 * dg.n if dg.vwgt is not None else 0)) + 48 * dg.n for dg in dgs]
    budget = max(fp) + min(fp)
    parts, res, info = _serve(J, jobs, dgs, 8, budget=budget)
    for (name, *_), p, r, (pa, sa) in zip(jobs, parts, res, alone):
        assert r["status"] == 0, name
        np.testing.assert_array_equal(p, pa, err_msg=name)
    # the budget binds: jobs were held back in the queue, admitted later than
    # submitted, and the footprint in use never exceeded the budget
    assert info["max_queued"] > 0
    assert any(r["t_admit_ms"] > r["t_submit_ms"] for r in res)
    assert 0 < info["max_in_use"] <= budget and info["hbm_in_use"] == 0
    import torch
    sv = J.Server(hbm_budget_bytes=min(fp) - 1, max_slots=2)
    try:
        with pytest.raises(J.JetError) as e:
            sv.submit(dgs[0], torch.empty(dgs[0].n, dtype=torch.int32, device="cuda"), 4)
        assert e.value.status == J.JET_ELIMIT
    finally:
        sv.close()


def test_server_matches_oracle(J):
    import torch
    from oracle import oracle as O
    jobs = [("grid32_k4", I.grid2d(32, 32), True, 4, 11),
            ("rmat11_k16", I.rmat(11, 8, 24), False, 16, 12),
            ("er_k3", I.small_random_graph(90, 0.08, 5, wmax=4, vwmax=2), False, 3, 13)]
    dgs = [J.to_device(g, unit_vwgt=unit, unit_adjwgt=unit) for _, g, unit, _, _ in jobs]
    parts, res, info = _serve(J, jobs, dgs, 3)
    for (name, g, unit, k, seed), p, r in zip(jobs, parts, res):
        exp = O.partition(g, k, seed=seed)
        np.testing.assert_array_equal(p, exp["part"], err_msg=name)
        assert r["cut"] == exp["cut"], name


def test_server_errors(J):
    import torch
    sv = J.Server(max_slots=2)
    try:
        g = I.grid2d(8, 8)
        dg = J.to_device(g)
        with pytest.raises(J.JetError) as e:
            sv.submit(dg, torch.empty(g.n, dtype=torch.int32, device="cuda"), 0)
        assert e.value.status == J.JET_EINVAL
        with pytest.raises(J.JetError) as e:
            sv.poll(12345)
        assert e.value.status == J.JET_EINVAL
        # a malformed graph fails its own job only
        bad_adj = dg.adjncy.clone()
        bad_adj[3] = g.n + 5
        bad = J.DeviceGraph(dg.xadj, bad_adj, dg.vwgt, dg.adjwgt)
        out_bad = torch.empty(g.n, dtype=torch.int32, device="cuda")
        out_ok = torch.empty(g.n, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()  # the server works on a stream of its own
        t_bad = sv.submit(bad, out_bad, 4)
        t_ok = sv.submit(dg, out_ok, 4, seed=3)
        rb = sv.wait(t_bad, 60000)
        assert rb["status"] == J.JET_EGRAPH
        r = sv.wait(t_ok, 60000)
        assert r["status"] == 0
        part, st, _ = J.partition(dg, 4, seed=3)
        np.testing.assert_array_equal(out_ok.cpu().numpy(), part.cpu().numpy())
    finally:
        sv.close()
