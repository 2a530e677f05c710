"""Parity of the largest single graph: R-MAT scale 22 (n = 4,194,304,
2m = 128,316,062, about 43% isolated vertices, hub rows of up to 163K
entries), edge factor 16, (a,b,c,d) = (0.57,0.19,0.19,0.05), edge weights
1..16, k = 256, lambda 3%, seed 2 -- the whole multilevel partition
(Algorithm 1 with Algorithms 3-5 and Jetrs on every level) through the call
bench.py times.

The expected values are the oracle's own run, stored by
tests/golden/make_rmat22_k256.py (which calls only oracle/ and the input
generator; the oracle takes minutes on one core): every per-iteration trace
record of every level (kind, counts, cut, largest part weight, best cut,
stall and weak-rebalance counters, partition digest), the final cut and
balance, the SHA-256 of the final partition and the parts of 4096 sampled
vertices. The graph itself is pinned by the SHA-256 of its CSR arrays.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np
import pytest

from paper_2304_13194_amd import inputs as I

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rmat22_k256.json")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _graph_sha256(g):
    h = hashlib.sha256()
    for arr, dt in ((g.xadj, "<i8"), (g.adjncy, "<i4"), (g.vwgt, "<i4"), (g.adjwgt, "<i4")):
        h.update(np.ascontiguousarray(arr, dtype=dt).tobytes())
    return h.hexdigest()


@pytest.fixture(scope="module")
def J():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_13194_amd import jet
    jet.lib()
    return jet


@pytest.fixture(scope="module")
def case():
    with open(GOLDEN) as f:
        gold = json.load(f)
    gd = gold["graph"]
    t0 = time.perf_counter()
    g = I.rmat(gd["scale"], gd["edge_factor"], gd["gen_seed"])
    _say(f"R-MAT scale {gd['scale']}: n={g.n} 2m={g.nnz} generated in {time.perf_counter() - t0:.1f} s")
    assert g.n == gd["n"] and g.nnz == gd["nnz"]
    assert _graph_sha256(g) == gd["sha256"], "the generator no longer draws the graph the oracle partitioned"
    return g, gold


def _check(part, st, tr, gold, label):
    assert st["levels"] == len(gold["level_sizes"]), label
    if tr is not None:
        assert len(tr) == len(gold["trace"]), label
        for a, b in zip(tr, gold["trace"]):
            assert a == b, f"{label}: gpu {a} != oracle {b}"
    ids = np.asarray(gold["sample_ids"], dtype=np.int64)
    np.testing.assert_array_equal(part[ids], np.asarray(gold["sample_parts"], dtype=np.int32),
                                  err_msg=f"{label}: sampled parts")
    assert hashlib.sha256(np.ascontiguousarray(part, dtype="<i4").tobytes()).hexdigest() == gold["part_sha256"], label
    assert st["cut"] == gold["cut"] and st["max_part_weight"] == gold["maxw"], label
    assert bool(st["balanced"]) == gold["balanced"] and st["o"] == gold["o"], label


@pytest.mark.timeout(900)
def test_rmat22_k256_partition_matches_oracle(J, case):
    """As timed (profiling flag, trace), then with graph replay and no trace:
    both equal the oracle's partition, and the cut and part weights
    recomputed from the returned partition equal the reported ones."""
    import torch
    g, gold = case
    dg = J.to_device(g)
    part, st, tr = J.partition(dg, gold["k"], seed=gold["seed"], flags=J.JET_F_PROFILE, trace_cap=1 << 16)
    torch.cuda.synchronize()
    part = part.cpu().numpy()
    _say(f"gpu (profiled): cut={st['cut']} iters={st['iters']} levels={st['levels']}")
    _check(part, st, tr, gold, "profiled")
    part2, st2, _ = J.partition(dg, gold["k"], seed=gold["seed"])
    torch.cuda.synchronize()
    _check(part2.cpu().numpy(), st2, None, gold, "graph replay")
    # independent recount from the CSR arrays
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.xadj))
    diff = part[src] != part[g.adjncy]
    cut = int(np.sum(g.adjwgt[diff].astype(np.int64))) // 2
    pw = np.bincount(part, weights=g.vwgt, minlength=gold["k"]).astype(np.int64)
    assert cut == st["cut"] and int(pw.max()) == st["max_part_weight"] and int(pw.sum()) == g.n
