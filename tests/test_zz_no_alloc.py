"""jet_refine_noalloc, the refinement entry point for callers that cannot
allocate, against jet_refine through the C ABI.

Both calls refine the same seeded start; the partition, every trace record,
the statistics and the part weights must be identical (integer work:
bit-exact). The calls run back to back on one context: a hub-row R-MAT
graph with edge weights (long rows in 1024-entry chunks), then a smaller
grid, then the R-MAT graph again, so a call that read anything the previous
call left in the shared scratch array would show here. The limits: k = 1,
JET_F_VALIDATE and JET_F_PROFILE are rejected, and a graph whose workspace
exceeds the array is rejected with JET_ELIMIT before any device work, its
partition untouched.
"""
import sys

import numpy as np
import pytest

from paper_2304_13194_amd import inputs as I

pytestmark = pytest.mark.gpu

STAT_KEYS = ("cut", "max_part_weight", "o", "sigma", "total_weight", "balanced", "iters", "lp_iters",
             "rw_iters", "rs_iters", "levels")


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


def _pair(J, g, k, seed, unit):
    import torch
    dg = J.to_device(g, unit_vwgt=unit, unit_adjwgt=unit)
    p0 = torch.from_numpy(I.random_partition(g.n, k, seed)).cuda()
    a = p0.clone()
    st_a, tr_a, pw_a = J.refine(dg, a, k, seed=seed, trace_cap=4096, part_weights=True)
    b = p0.clone()
    pw_b = torch.full((k,), -1, dtype=torch.int64, device="cuda")
    st_b, tr_b, _ = J.refine_noalloc(dg, b, k, seed=seed, trace_cap=4096, part_weights=pw_b)
    torch.cuda.synchronize()
    _say(f"  n={g.n} 2m={g.nnz} k={k}: iters {st_a['iters']} / {st_b['iters']}, cut {st_a['cut']} / {st_b['cut']}")
    assert torch.equal(a, b)
    assert tr_a == tr_b and len(tr_a) == st_a["iters"]
    for key in STAT_KEYS:
        assert st_a[key] == st_b[key], key
    assert torch.equal(pw_a, pw_b)


def test_noalloc_matches_refine_back_to_back(J):
    big = I.rmat(14, 16, 6)
    assert int(np.diff(big.xadj).max()) > 1024  # long rows take the chunk kernels
    _say("R-MAT scale 14 (weights), k = 64")
    _pair(J, big, 64, 11, unit=False)
    _say("grid 64x64 (unit weights), k = 4")
    _pair(J, I.grid2d(64, 64), 4, 12, unit=True)
    _say("R-MAT scale 14 again, k = 37")
    _pair(J, big, 37, 13, unit=False)


def test_noalloc_limits(J):
    import torch
    g = I.grid2d(16, 16)
    dg = J.to_device(g)
    p = torch.zeros(g.n, dtype=torch.int32, device="cuda")
    with pytest.raises(J.JetError) as e:
        J.refine_noalloc(dg, p, 1)
    assert e.value.status == J.JET_EINVAL
    for fl in (J.JET_F_VALIDATE, J.JET_F_PROFILE):
        with pytest.raises(J.JetError) as e:
            J.refine_noalloc(dg, p, 4, flags=fl)
        assert e.value.status == J.JET_EINVAL
    # 5M isolated vertices need about 165 MB of workspace: over the array
    n = 5_000_000
    big = J.DeviceGraph(torch.zeros(n + 1, dtype=torch.int64, device="cuda"),
                        torch.zeros(0, dtype=torch.int32, device="cuda"), None, None)
    part = torch.full((n,), 3, dtype=torch.int32, device="cuda")
    with pytest.raises(J.JetError) as e:
        J.refine_noalloc(big, part, 8)
    assert e.value.status == J.JET_ELIMIT
    torch.cuda.synchronize()
    assert bool((part == 3).all())
