"""GPU parity of the refinement kernels against the CPU oracle.

Each case runs through the C ABI (via the thin binding) and is compared with
the oracle element by element: Jetlp step outputs (P_d, F, conn(v, P_s), X,
F2, M), rebalancing step outputs (destination, loss, slot), and the full
refinement loop (every per-iteration trace field, including the partition
digest, plus P_best). Integer work: the bar is bit-exact equality.
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


def stars(sizes, seed=5):
    """Disjoint stars (centre degrees = sizes) joined by a sparse random ring of
    leaves, so long rows cross chunk boundaries at 1024-entry multiples."""
    us, vs, base = [], [], 0
    for m in sizes:
        us.append(np.full(m, base, np.int64))
        vs.append(np.arange(base + 1, base + m + 1, dtype=np.int64))
        base += m + 1
    n = base
    leaves = np.array([v for v in range(n) if v not in set(np.cumsum([0] + [m + 1 for m in sizes[:-1]]))], np.int64)
    order = leaves[np.argsort(I.stream(seed, np.arange(leaves.size, dtype=np.uint64)), kind="stable")]
    a, b = order[::7], np.roll(order[::7], 1)
    keep = a != b
    us.append(np.minimum(a[keep], b[keep]))
    vs.append(np.maximum(a[keep], b[keep]))
    u = np.concatenate(us)
    v = np.concatenate(vs)
    key = np.unique(u * n + v)
    return I.csr_from_edges(n, key // n, key % n)


def _reweight(g, lo, hi, seed):
    """g with symmetric edge weights drawn from [lo, hi)."""
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.xadj))
    keep = src < g.adjncy
    u, v = src[keep], g.adjncy[keep].astype(np.int64)
    w = (lo + I.uniform_below(I.stream(seed, np.arange(u.size, dtype=np.uint64)), hi - lo)).astype(np.int32)
    return I.csr_from_edges(g.n, u, v, w)


def cases():
    """(name, graph, k, level) covering every kernel role."""
    out = [
        ("grid64_k4", I.grid2d(64, 64), 4, 0),
        ("stencil12_k8", I.stencil27(12, 12, 12), 8, 0),
        ("stencil12_k8_l2", I.stencil27(12, 12, 12), 8, 2),
        ("rmat12_k32_w", I.rmat(12, 8, 5), 32, 0),
        ("rmat14_k64_hubs", I.rmat(14, 16, 6), 64, 1),
        ("rmat12_k200", I.rmat(12, 8, 9), 200, 0),
        ("rmat12_k600", I.rmat(12, 8, 7), 600, 0),
        ("rmat12_k5000", I.rmat(12, 8, 8), 5000, 0),
        ("star3000_k3", star(3000), 3, 0),
        ("stars_chunks_k4", stars([1024, 1025, 2048, 2049, 4100]), 4, 0),
        # rows of several 4096-entry chunks (full and ragged last chunks)
        ("stars_multichunk_k16", stars([4096, 4097, 8192, 9000, 13001]), 16, 0),
        # long rows at k >= 4096 (one 16 KiB or 64 KiB chunk table per block)
        ("stars_long_k5000", stars([1025, 4100, 9000]), 5000, 0),
        ("stars_long_k16384", stars([1025, 4100]), 16384, 0),
        ("rgg3000_k16", I.rgg(3000, 9), 16, 0),
        # gains beyond the afterburner's 16-bit packed F: equal weights make
        # many equal F above the bound (the full F breaks those ties), and
        # large random weights spread F on both sides of it
        ("grid48_w40000_k4", _reweight(I.grid2d(48, 48), 40000, 40001, 1), 4, 0),
        ("rmat12_w20k_70k_k200_l1", _reweight(I.rmat(12, 8, 9), 20000, 70000, 2), 200, 1),
        ("rmat12_w20k_70k_k300", _reweight(I.rmat(12, 8, 9), 20000, 70000, 3), 300, 0),
        # the last k whose part ids fit a byte (compact Jetlp records, part id 255
        # in use) and the first that takes the full records
        ("rmat12_w20k_70k_k256", _reweight(I.rmat(12, 8, 9), 20000, 70000, 4), 256, 0),
        ("rmat12_w20k_70k_k257", _reweight(I.rmat(12, 8, 9), 20000, 70000, 4), 257, 0),
    ]
    for s in range(6):
        g = I.small_random_graph(30 + 11 * s, 0.15, 600 + s, wmax=1 + s % 5, vwmax=1 + s % 3)
        out.append((f"er{s}", g, 2 + s, s % 2))
    return out


CASES = cases()


def _locks(n, seed):
    return (I.stream(seed, np.arange(n, dtype=np.uint64)) % np.uint64(7) == 0).astype(np.uint8)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_lp_step_parity(J, O, case):
    import torch
    name, g, k, level = case
    _say(f"lp_step {name} n={g.n} nnz={g.nnz} k={k}")
    dg = J.to_device(g)
    for trial in range(2):
        P = I.random_partition(g.n, k, 100 + trial)
        L = _locks(g.n, 200 + trial) if trial else np.zeros(g.n, np.uint8)
        exp = O.jetlp(g, P, L, k, level=level)
        got = J.lp_step(dg, torch.from_numpy(P).cuda(), torch.from_numpy(L).cuda(), k, level=level)
        for key in ("pd", "F", "conn_s", "F2"):
            np.testing.assert_array_equal(got[key].cpu().numpy(), exp[key], err_msg=f"{name} {key}")
        np.testing.assert_array_equal(got["inX"].cpu().numpy().astype(bool), exp["inX"], err_msg=f"{name} inX")
        np.testing.assert_array_equal(got["move"].cpu().numpy().astype(bool), exp["move"], err_msg=f"{name} move")


def _skewed(g, k, seed):
    x = I.stream(seed, np.arange(g.n, dtype=np.uint64))
    y = I.stream(seed + 1, np.arange(g.n, dtype=np.uint64))
    return np.where(I.uniform_below(x, 3) == 0, I.uniform_below(y, k), I.uniform_below(y, max(1, k // 3)))\
        .astype(np.int32)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_rebalance_step_parity(J, O, case):
    import torch
    name, g, k, level = case
    _say(f"rebalance_step {name} n={g.n} k={k}")
    dg = J.to_device(g)
    P = _skewed(g, k, 300)
    for kind in (J.KIND_RW, J.KIND_RS):
        for t in (0, 5):
            exp = O.rebalance(g, P, kind, t, k, level=level, seed=77)
            got = J.rebalance_step(dg, torch.from_numpy(P).cuda(), kind, t, k, level=level, seed=77)
            for key in ("dest", "loss", "slot"):
                np.testing.assert_array_equal(got[key].cpu().numpy(), exp[key], err_msg=f"{name} {kind} {t} {key}")


def _compare_refine(J, O, g, k, P0, name, level=0, seed=0, bmax=None, **kw):
    import torch
    _say(f"refine {name} n={g.n} k={k} level={level}")
    okw = dict(kw)
    gkw = dict(kw)
    if bmax is not None:
        okw["bmax"] = bmax
        gkw["weak_rebalance_iters"] = -1 if bmax == 0 else bmax
    exp = O.refine(g, P0, k, level=level, seed=seed, **okw)
    dg = J.to_device(g)
    part = torch.from_numpy(P0.copy()).cuda()
    st, tr, pw = J.refine(dg, part, k, trace_cap=10000, part_weights=True, level=level, seed=seed, **gkw)
    assert st["iters"] == exp.iters, name
    assert len(tr) == len(exp.trace)
    for a, b in zip(tr, exp.trace):
        assert a == b, f"{name}: gpu {a} != oracle {b}"
    np.testing.assert_array_equal(part.cpu().numpy(), exp.part, err_msg=name)
    assert st["cut"] == exp.cut and st["max_part_weight"] == exp.maxw and bool(st["balanced"]) == exp.balanced
    w = np.bincount(exp.part, weights=g.vwgt, minlength=k).astype(np.int64)
    np.testing.assert_array_equal(pw.cpu().numpy(), w)
    return st


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_refine_parity_random_start(J, O, case):
    name, g, k, level = case
    P0 = I.random_partition(g.n, k, 400)
    _compare_refine(J, O, g, k, P0, name, level=level, seed=11)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_refine_parity_skewed_start(J, O, case):
    """Imbalanced start: exercises Jetrw, Jetrs and the least-imbalance best."""
    name, g, k, level = case
    _compare_refine(J, O, g, k, _skewed(g, k, 500), name + "_skew", level=level, seed=12)


def test_refine_parity_options(J, O):
    g = I.grid2d(64, 64)
    P0 = I.random_partition(g.n, 4, 1)
    _compare_refine(J, O, g, 4, P0, "grid_c34", c=(3, 4))
    _compare_refine(J, O, g, 4, P0, "grid_phi", phi=(99, 100), stall_limit=5)
    _compare_refine(J, O, g, 4, _skewed(g, 4, 3), "grid_rs_only", bmax=0)
    _compare_refine(J, O, g, 4, _skewed(g, 4, 3), "grid_rw_5", bmax=5)
    _compare_refine(J, O, g, 8, _skewed(g, 8, 3), "grid_lam10", lambda_ppm=100000)


def test_refine_iteration_vectors_cfg1(J, O):
    """64x64 grid, k = 4, lambda 3%, seeded random start: P_iter after every
    iteration equals the oracle's (full vectors)."""
    import torch
    g = I.grid2d(64, 64)
    P0 = I.random_partition(g.n, 4, I.subseed(1, 1))
    exp_all = O.refine(g, P0, 4)
    dg = J.to_device(g)
    for t in range(1, exp_all.iters + 1):
        exp = O.refine(g, P0, 4, max_iters=t)
        part = torch.from_numpy(P0.copy()).cuda()
        J.refine(dg, part, 4, max_iters=t, flags=J.JET_F_RETURN_ITER)
        np.testing.assert_array_equal(part.cpu().numpy(), exp.iter_part, err_msg=f"t={t}")


def test_refine_deterministic(J):
    import torch
    g = I.rmat(13, 12, 21)
    dg = J.to_device(g)
    P0 = torch.from_numpy(I.random_partition(g.n, 48, 5)).cuda()
    outs = []
    for _ in range(3):
        p = P0.clone()
        st, tr, _ = J.refine(dg, p, 48, trace_cap=1000)
        outs.append((p.cpu().numpy(), tr))
    for p, tr in outs[1:]:
        np.testing.assert_array_equal(p, outs[0][0])
        assert tr == outs[0][1]


def test_refine_unit_weight_pointers(J, O):
    """NULL vwgt / adjwgt (unit weights) give the same result as explicit ones."""
    import torch
    g = I.stencil27(10, 10, 10)
    P0 = I.random_partition(g.n, 6, 9)
    exp = O.refine(g, P0, 6)
    dg = J.to_device(g, unit_vwgt=True, unit_adjwgt=True)
    part = torch.from_numpy(P0.copy()).cuda()
    J.refine(dg, part, 6)
    np.testing.assert_array_equal(part.cpu().numpy(), exp.part)


def test_refine_edge_cases(J, O):
    import torch
    # k = 1: all zeros
    g = I.grid2d(8, 8)
    dg = J.to_device(g)
    p = torch.from_numpy(I.random_partition(g.n, 3, 1)).cuda()
    st, _, _ = J.refine(dg, p, 1)
    assert int(p.abs().sum()) == 0 and st["cut"] == 0
    # part id out of range -> JET_EPART, part untouched
    bad = torch.from_numpy(I.random_partition(g.n, 3, 1)).cuda()
    bad[5] = 7
    before = bad.clone()
    with pytest.raises(J.JetError) as e:
        J.refine(dg, bad, 3)
    assert e.value.status == J.JET_EPART
    assert torch.equal(bad, before)
    # k < 1 -> JET_EINVAL; k too large -> JET_ELIMIT
    with pytest.raises(J.JetError) as e:
        J.refine(dg, p, 0)
    assert e.value.status == J.JET_EINVAL
    with pytest.raises(J.JetError) as e:
        J.refine(dg, p, 20000)
    assert e.value.status == J.JET_ELIMIT
    # self-loop -> JET_EGRAPH (cheap check), asymmetric -> JET_EGRAPH with validation
    adj = dg.adjncy.clone()
    adj[0] = 0
    dg2 = J.DeviceGraph(dg.xadj, adj, None, None)
    with pytest.raises(J.JetError) as e:
        J.refine(dg2, p.clone(), 3)
    assert e.value.status == J.JET_EGRAPH
    adj = dg.adjncy.clone()
    adj[0] = 9 if int(adj[0]) != 9 else 10
    dg3 = J.DeviceGraph(dg.xadj, adj, None, None)
    with pytest.raises(J.JetError) as e:
        J.refine(dg3, p.clone(), 3, flags=J.JET_F_VALIDATE)
    assert e.value.status == J.JET_EGRAPH
    # graph with only isolated vertices
    gi = I.csr_from_edges(50, np.zeros(0, np.int64), np.zeros(0, np.int64))
    P0 = np.zeros(50, np.int32)
    _compare_refine(J, O, gi, 4, P0, "isolated_only")


# Jetlp ablations (Section 7.1, Component Effectiveness, Table lp_versions): (name, c, flags)
def _ablations(J):
    NL, NA = J.JET_F_LP_NO_LOCKS, J.JET_F_LP_NO_AFTERBURNER
    return [("baseline", (0, 1), NL | NA), ("locks", (0, 1), NA), ("weak_afterburner", (0, 1), NL),
            ("full_afterburner", None, NL), ("full", None, 0)]


ABL_CASES = [c for c in CASES if c[0] in ("grid64_k4", "rmat12_k32_w", "stencil12_k8_l2", "rmat14_k64_hubs",
                                           "stars_chunks_k4", "er3")]


@pytest.mark.parametrize("case", ABL_CASES, ids=[c[0] for c in ABL_CASES])
def test_refine_ablation_parity(J, O, case):
    name, g, k, level = case
    for vname, c, flags in _ablations(J):
        kw = dict(flags=flags)
        if c is not None:
            kw["c"] = c
        _compare_refine(J, O, g, k, I.random_partition(g.n, k, 700), f"{name}_{vname}", level=level, seed=13, **kw)


@pytest.mark.parametrize("case", ABL_CASES, ids=[c[0] for c in ABL_CASES])
def test_lp_step_no_afterburner_parity(J, O, case):
    import torch
    name, g, k, level = case
    dg = J.to_device(g)
    P = I.random_partition(g.n, k, 101)
    L = _locks(g.n, 201)
    for c in ((0, 1), None):
        kw = {} if c is None else dict(c=c)
        exp = O.jetlp(g, P, L, k, level=level, flags=O.F_NO_AFTERBURNER, **kw)
        got = J.lp_step(dg, torch.from_numpy(P).cuda(), torch.from_numpy(L).cuda(), k, level=level,
                        flags=J.JET_F_LP_NO_AFTERBURNER, **kw)
        for key in ("pd", "F", "conn_s", "F2"):
            np.testing.assert_array_equal(got[key].cpu().numpy(), exp[key], err_msg=f"{name} {key}")
        np.testing.assert_array_equal(got["move"].cpu().numpy().astype(bool), exp["move"], err_msg=name)



@pytest.mark.parametrize("weights", ["null", "explicit_unit", "random"])
def test_refine_large_mesh_split_launch(J, O, weights):
    """A graph of 2^18 vertices whose rows all have at most 32 entries: the
    gain and loss passes run in launches of their own, with two rows in
    flight per lane group when edge weights are NULL (unit) and one row per
    round otherwise. Start: z-slabs with the last part three slabs wide and
    2% of the vertices reassigned at random (Jetlp, Jetrw and Jetrs all run);
    k = 16, against the oracle."""
    import torch
    g = I.stencil27(64, 64, 64)
    if weights == "random":
        # symmetric weights 1..7 from a hash of the two endpoints
        src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.xadj))
        lo = np.minimum(src, g.adjncy).astype(np.uint64)
        hi = np.maximum(src, g.adjncy).astype(np.uint64)
        h = (lo * np.uint64(2654435761) + hi * np.uint64(40503)) % np.uint64(7)
        g = I.Graph(g.xadj, g.adjncy, g.vwgt, (1 + h).astype(np.int32), "stencil64_weighted")
    k = 16
    rng = np.random.default_rng(3)
    P0 = np.minimum((np.arange(g.n) * (k + 2)) // g.n, k - 1).astype(np.int32)
    idx = rng.choice(g.n, g.n // 50, replace=False)
    P0[idx] = rng.integers(0, k, idx.size)
    exp = O.refine(g, P0, k, seed=5)
    assert {t["kind"] for t in exp.trace} == {1, 2, 3}
    unit = weights == "null"
    dg = J.to_device(g, unit_vwgt=unit, unit_adjwgt=unit)
    part = torch.from_numpy(P0.copy()).cuda()
    st, tr, _ = J.refine(dg, part, k, trace_cap=10000, seed=5)
    assert st["iters"] == exp.iters
    assert len(tr) == len(exp.trace)
    for a, b in zip(tr, exp.trace):
        assert a == b, f"{weights}: gpu {a} != oracle {b}"
    np.testing.assert_array_equal(part.cpu().numpy(), exp.part)
    assert st["cut"] == exp.cut and st["max_part_weight"] == exp.maxw


def _heavy(g, seed, lo=1 << 24, hi=1 << 25):
    """g with symmetric edge weights drawn from [lo, hi): its total edge weight
    is far above 2^31 while every weighted degree stays below it."""
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.xadj))
    keep = src < g.adjncy
    u, v = src[keep], g.adjncy[keep].astype(np.int64)
    w = (lo + I.uniform_below(I.stream(seed, np.arange(u.size, dtype=np.uint64)), hi - lo)).astype(np.int32)
    return I.csr_from_edges(g.n, u, v, w)


def test_refine_large_total_edge_weight(J, O):
    """Single-level refinement only needs every weighted degree below 2^31
    (connectivities, gains, losses are int32; cuts and part weights int64):
    a grid whose total edge weight is about 2^36 matches the oracle (int64
    throughout) step by step, loop by loop and in a batch; a vertex whose
    weighted degree reaches 2^31 is rejected, and multilevel partitioning
    keeps the total-weight limit (coarse edge weights are int32 sums)."""
    import torch
    g = _heavy(I.grid2d(48, 48), 31)
    total = int(g.adjwgt.astype(np.int64).sum())
    wdeg = np.add.reduceat(g.adjwgt.astype(np.int64), g.xadj[:-1])
    assert total >= 2 ** 31 and int(wdeg.max()) < 2 ** 31
    k = 4
    _compare_refine(J, O, g, k, I.random_partition(g.n, k, 41), "heavy_random", seed=3)
    _compare_refine(J, O, g, k, _skewed(g, k, 42), "heavy_skewed", seed=4)
    dg = J.to_device(g)
    P = I.random_partition(g.n, k, 43)
    L = _locks(g.n, 44)
    exp = O.jetlp(g, P, L, k)
    got = J.lp_step(dg, torch.from_numpy(P).cuda(), torch.from_numpy(L).cuda(), k)
    for key in ("pd", "F", "conn_s", "F2"):
        np.testing.assert_array_equal(got[key].cpu().numpy(), exp[key], err_msg=key)
    S = _skewed(g, k, 45)
    for kind in (J.KIND_RW, J.KIND_RS):
        exp = O.rebalance(g, S, kind, 1, k, seed=5)
        got = J.rebalance_step(dg, torch.from_numpy(S).cuda(), kind, 1, k, seed=5)
        for key in ("dest", "loss", "slot"):
            np.testing.assert_array_equal(got[key].cpu().numpy(), exp[key], err_msg=f"{kind} {key}")
    # in a batch with a second heavy graph: each equals its oracle run
    g2 = _heavy(I.grid2d(40, 56), 32)
    graphs = [g, g2]
    p0 = [I.random_partition(x.n, k, 46 + i) for i, x in enumerate(graphs)]
    parts = [torch.from_numpy(p.copy()).cuda() for p in p0]
    stats, _ = J.refine_batch([J.to_device(x) for x in graphs], parts, [dict(k=k, seed=6)] * 2)
    for x, p, q, st in zip(graphs, p0, parts, stats):
        e = O.refine(x, p, k, seed=6)
        np.testing.assert_array_equal(q.cpu().numpy(), e.part)
        assert st["cut"] == e.cut and st["cut"] >= 2 ** 31
    # a weighted degree of 2^31 or more: rejected before any refinement
    star3 = I.csr_from_edges(4, np.zeros(3, np.int64), np.arange(1, 4), np.full(3, 2 ** 30, np.int32))
    p = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(J.JetError) as e:
        J.refine(J.to_device(star3), p, 2)
    assert e.value.status == J.JET_EOVERFLOW
    with pytest.raises(J.JetError) as e:
        J.partition(dg, k)
    assert e.value.status == J.JET_EOVERFLOW


def test_refine_async(J, O):
    """JET_F_ASYNC: the call returns once the iterations are enqueued; after
    the stream completes, partition, part weights, stats and every trace
    record equal the blocking call's (and the oracle's)."""
    import torch
    g = I.rmat(13, 12, 22)
    k = 24
    dg = J.to_device(g)
    P0 = I.random_partition(g.n, k, 51)
    a = torch.from_numpy(P0.copy()).cuda()
    st_a, tr_a, pw_a = J.refine(dg, a, k, seed=7, trace_cap=1000, part_weights=True, max_iters=300)
    b = torch.from_numpy(P0.copy()).cuda()
    h = J.refine_async(dg, b, k, 300, seed=7, trace_cap=1000, part_weights=True)
    st_b, tr_b, pw_b = h.wait()
    assert torch.equal(a, b) and torch.equal(pw_a, pw_b)
    assert tr_a == tr_b and len(tr_b) == st_b["iters"] == st_b["trace_total"]
    for key in ("cut", "max_part_weight", "o", "sigma", "balanced", "iters", "lp_iters", "rw_iters", "rs_iters"):
        assert st_a[key] == st_b[key], key
    exp = O.refine(g, P0, k, seed=7, max_iters=300)
    np.testing.assert_array_equal(b.cpu().numpy(), exp.part)
    assert tr_b == exp.trace
    # a cap below the natural end: the loop stops at the cap, as blocking
    c = torch.from_numpy(P0.copy()).cuda()
    st_c, tr_c, _ = J.refine_async(dg, c, k, 5, seed=7, trace_cap=1000).wait()
    exp5 = O.refine(g, P0, k, seed=7, max_iters=5)
    assert st_c["iters"] == 5 and tr_c == exp5.trace
    np.testing.assert_array_equal(c.cpu().numpy(), exp5.part)
    # rejected: no cap, with profiling, and on the multilevel and batch calls
    for kw in (dict(max_iters=0), dict(max_iters=10, flags=J.JET_F_PROFILE)):
        with pytest.raises(J.JetError) as e:
            J.refine(dg, torch.from_numpy(P0.copy()).cuda(), k, flags=J.JET_F_ASYNC | kw.pop("flags", 0), **kw)
        assert e.value.status == J.JET_EINVAL
    with pytest.raises(J.JetError) as e:
        J.partition(dg, k, flags=J.JET_F_ASYNC, max_iters=10)
    assert e.value.status == J.JET_EINVAL
    with pytest.raises(J.JetError) as e:
        J.refine_batch([dg], [torch.from_numpy(P0.copy()).cuda()], [dict(k=k, flags=J.JET_F_ASYNC, max_iters=10)])
    assert e.value.status == J.JET_EINVAL


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_conn_table_parity(J, O, case):
    """Section 4.3's persistent connectivity table (JET_F_CONN_TABLE): the
    Jetlp and rebalancing step outputs from rows built once, and the whole
    refinement loop with rows kept up to date by Algorithm 6 (decrement,
    increment with inserts, rebuilds of full rows, whole rebuilds after large
    move sets), equal the oracle's, which recomputes connectivity from
    scratch."""
    import torch
    name, g, k, level = case
    TF = J.JET_F_CONN_TABLE
    dg = J.to_device(g)
    P = I.random_partition(g.n, k, 100)
    L = _locks(g.n, 201)
    exp = O.jetlp(g, P, L, k, level=level)
    got = J.lp_step(dg, torch.from_numpy(P).cuda(), torch.from_numpy(L).cuda(), k, level=level, flags=TF)
    for key in ("pd", "F", "conn_s", "F2"):
        np.testing.assert_array_equal(got[key].cpu().numpy(), exp[key], err_msg=f"{name} {key}")
    S = _skewed(g, k, 300)
    for kind in (J.KIND_RW, J.KIND_RS):
        exp = O.rebalance(g, S, kind, 3, k, level=level, seed=77)
        got = J.rebalance_step(dg, torch.from_numpy(S).cuda(), kind, 3, k, level=level, seed=77, flags=TF)
        for key in ("dest", "loss", "slot"):
            np.testing.assert_array_equal(got[key].cpu().numpy(), exp[key], err_msg=f"{name} {kind} {key}")
    _compare_refine(J, O, g, k, I.random_partition(g.n, k, 400), name + "_table", level=level, seed=11, flags=TF)
    _compare_refine(J, O, g, k, _skewed(g, k, 500), name + "_table_skew", level=level, seed=12, flags=TF)


def test_conn_table_partition_parity(J, O):
    """Multilevel partitions with the table on every level equal the oracle's."""
    import torch
    for name, g, k, unit in (("stencil16_k8", I.stencil27(16, 16, 16), 8, True),
                             ("rmat14_k64", I.rmat(14, 16, 6), 64, False),
                             ("grid96_k5", I.grid2d(96, 96), 5, True)):
        dg = J.to_device(g, unit_vwgt=unit, unit_adjwgt=unit)
        part, st, tr = J.partition(dg, k, seed=3, flags=J.JET_F_CONN_TABLE, trace_cap=1 << 14)
        exp = O.partition(g, k, seed=3, trace_cap=1 << 14)
        assert tr == exp["trace"], name
        np.testing.assert_array_equal(part.cpu().numpy(), exp["part"], err_msg=name)


@pytest.mark.parametrize("k", [64, 256, 257, 5000])
def test_gather_ceiling_runs_and_rejects(J, k):
    """jet_gather_ceiling (byte parts for k <= 256, else 16-bit) times a pass
    and rejects bad arguments before any device work."""
    import torch
    g = I.rmat(12, 8, 3)
    _say(f"gather ceiling rmat12 k={k}")
    dg = J.to_device(g)
    part = torch.from_numpy(I.random_partition(g.n, k, 1)).cuda()
    ms = J.gather_ceiling(dg, part, k, reps=2)
    assert ms > 0
    with pytest.raises(J.JetError) as e:
        J.gather_ceiling(dg, part, 0, reps=2)
    assert e.value.status == J.JET_EINVAL
    with pytest.raises(J.JetError) as e:
        J.gather_ceiling(dg, part, 16385, reps=2)
    assert e.value.status == J.JET_ELIMIT
