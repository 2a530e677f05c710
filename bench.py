"""Benchmark: Jet refinement on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload rmat22|stencil128|grid64]
                    [--secondary stencil128|none] [--no-cpu-baseline] [--no-batch] [--no-serve]
                    [--no-ablations] [--serve-jobs N] [--serve-warmup N] [--serve-budget-gb G]
                    [--serve-slots S]

A step is one full multilevel partition (Algorithm 1: heavy-edge coarsening,
seeded random coarsest partition, Jet refinement of every level, i.e. every
row of the refinement hot path) of a device-resident synthetic graph. The
default workload is the largest single graph: an R-MAT power-law graph of
scale 22 (4,194,304 vertices, 128,316,062 CSR entries, edge factor 16,
(a,b,c,d) = (0.57,0.19,0.19,0.05), edge weights 1..16), k = 256,
lambda = 3%. The 128^3 27-point stencil mesh (k = 64, unit weights) is
measured the same way as a secondary line.

Prints one JSON line:
  value        edges traversed by Jet iterations per second of step time:
               sum over the refinement iterations of all levels of that
               level's CSR entries (2m), divided by the whole step's wall
               time (coarsening and set-up included)
  roofline     the connectivity/gain pass of the finest level's Jetlp
               iterations (every launch of the pass, between HIP events on
               the library's stream): algorithmic bytes per pass / average
               pass time, against 8 TB/s HBM and against a device copy
               timed in the same run
  cpu_baseline the CPU oracle on this host, same unit: a bounded sample of
               the same workload (R-MAT: the oracle's refinement of the
               finest level from a seeded random partition for a fixed
               number of iterations, whose result the GPU reproduces)
  secondary    the same measurement on the stencil mesh (full oracle
               partition as its CPU baseline)
  batch        512 random geometric graphs refined in one jet_refine_batch
               call vs one jet_refine call per graph (graphs/s, identical
               partitions required), and the oracle on one core and on all
  serving      Poisson arrivals of partition jobs (grids and R-MAT graphs,
               each job drawn on its own) into jet_server under an HBM
               budget: p50 / p99 latency and graphs/s per arrival rate, vs
               partitioning the same jobs one at a time
  ablations    Jetlp variants (baseline synchronous LP, +locks, +weak or
               full afterburner, full Jetlp), phi 0.99 / 0.999 / 0.9999,
               two-hop coarsening and the graph-growing start: cut and
               partition time per variant
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per finest-level Jetlp gain pass from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs (each calibrated by a plain 2^28-byte copy), valid only for
# the kernel source they were taken on (profiles/gain_pass_rmat22_k256.md,
# profiles/k_gain_stencil128_k64.md).
TRAFFIC = {
    "rmat22": dict(src_sha256="25615504a2741f898dd681d4171dc5fb801f475f458a2c1094e1296eff410c05",
                   fetch=1876883518, write=68820405, fetch_factor=1.9997, write_factor=1.0),
    "stencil128": dict(src_sha256="25615504a2741f898dd681d4171dc5fb801f475f458a2c1094e1296eff410c05",
                       fetch=249036138, write=9872254, fetch_factor=1.9997, write_factor=1.0),
}


def measured_traffic(workload):
    """Bytes per pass, or None when none were taken or the kernel changed since."""
    import hashlib
    t = TRAFFIC.get(workload)
    if t is None:
        return None, None
    src = os.path.join(ROOT, "paper_2304_13194_amd", "csrc", "jet_refine.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if sha != t["src_sha256"]:
        return None, None
    return t["fetch"] + t["write"], t

WORKLOADS = {
    # R-MAT scale 22, edge factor 16, weights in [1, 16], k = 256
    "rmat22": dict(kind="rmat", scale=22, ef=16, k=256, unit=False,
                   label="R-MAT scale 22 (edge factor 16, a,b,c,d = 0.57,0.19,0.19,0.05)",
                   gain_kernels="k_rows<8, 4, false, 5>: rows of at most 8 entries one per lane, up to 64 in "
                                "groups of 8 lanes; k_gain<false, 2, 8, 4, 1>: 65..1024 one wave each; "
                                "k_lconn<false, false> + k_lgain_fin<false>: longer rows in 4096-entry chunks, one "
                                "block each, then a finishing launch"),
    # full multilevel partition of the 128^3 27-point mesh, k = 64
    "stencil128": dict(kind="stencil", side=128, k=64, unit=True,
                       label="27-point stencil 128^3",
                       gain_kernels="k_gain<false, 1, 4, 8, 1>: every row has at most 32 entries"),
    # 64 x 64 grid, k = 4
    "grid64": dict(kind="grid", side=64, k=4, unit=True, label="2-D grid 64x64",
                   gain_kernels="small-row lane groups"),
}


def make_graph(w):
    from paper_2304_13194_amd import inputs as I
    if w["kind"] == "stencil":
        s = w["side"]
        return I.stencil27(s, s, s)
    if w["kind"] == "rmat":
        return I.rmat(w["scale"], w["ef"], 3)
    return I.grid2d(w["side"], w["side"])


def load_or_make_graph(w, name, cache_dir):
    import numpy as np
    from paper_2304_13194_amd import inputs as I
    path = os.path.join(cache_dir, f"{name}.npz") if cache_dir else None
    if path and os.path.exists(path):
        z = np.load(path)
        return I.Graph(z["xadj"], z["adjncy"], z["vwgt"], z["adjwgt"], name)
    g = make_graph(w)
    if path:
        os.makedirs(cache_dir, exist_ok=True)
        np.savez(path, xadj=g.xadj, adjncy=g.adjncy, vwgt=g.vwgt, adjwgt=g.adjwgt)
    return g


def gain_bytes(entries, rows, vertices, weighted, listed=True, compact=False, in_x=0):
    """Algorithmic bytes of a connectivity/gain pass.

    Per CSR entry of an unlocked row: 4 B neighbour id (+4 B edge weight when
    weights are passed). Per unlocked row: 8 B row offsets, 4 B for its part
    id gathered by neighbours (counted once). Per visited vertex: 4 B list
    entry (none when every vertex is in the small-row class, whose list is
    then the identity and is not read), 4 B own part, 4 B lock stamp, and the
    record written: 8 B, or, when every part id fits a byte (compact), the
    4 B compact record plus the 4 B full F of each of the in_x vertices of X.
    """
    per_vertex = (4 if listed else 0) + 8 + (4 if compact else 8)
    return entries * (8 if weighted else 4) + rows * 12 + vertices * per_vertex + (4 * in_x if compact else 0)


# ------------------------------------------------------------ input makers --
# (module-level so a process pool can run them)

def _gen_rgg(args):
    from paper_2304_13194_amd import inputs as I
    n, seed = args
    return I.rgg(n, seed)


def _gen_pool_graph(spec):
    from paper_2304_13194_amd import inputs as I
    return I.serve_pool_graph(spec)


def _oracle_refine_job(args):
    """One RGG of the batch: generate it (not timed), then time the oracle's
    refinement of it from its seeded start. Runs in a worker process."""
    import time as _t
    from oracle import oracle as O
    from paper_2304_13194_amd import inputs as I
    out = []
    for n, k, s in args:
        g = I.rgg(n, s)
        p0 = I.random_partition(g.n, k, s)
        t0 = _t.perf_counter()
        O.refine(g, p0, k, seed=s)
        out.append(_t.perf_counter() - t0)
    return out


def _worker_init():
    """Generator and oracle workers run one thread each, so that they never
    compete with the thread that launches the timed kernels."""
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        import torch
        torch.set_num_threads(1)
    except ImportError:
        pass


def host_info():
    """CPU model and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count()
    return {"cpu_model": model, "nproc": ncpu}


def pool_workers():
    # the GPU machine grants one GPU's share of its host: at most 16 workers
    return max(1, min(16, host_info()["nproc"] or 1))


# -------------------------------------------------------------- sub-benches --

def copy_ceiling(reps=20, nbytes=1 << 30):
    """A plain device-to-device copy of `nbytes` (read + write), timed with HIP
    events on torch's stream: the measured HBM ceiling of this GPU."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"GBs": 2 * nbytes / (ms * 1e-3) / 1e9, "ms": ms, "bytes_read_plus_written": 2 * nbytes,
            "kernel": "torch copy_ of a 1 GiB int32 tensor"}


def measure_workload(J, name, g, w, seed, steps, warmup, ceiling):
    """Timed multilevel partitions of one device-resident graph."""
    import numpy as np
    import torch
    k = w["k"]
    dg = J.to_device(g, unit_vwgt=w["unit"], unit_adjwgt=w["unit"])
    torch.cuda.synchronize()
    # level sizes (n, 2m) of the hierarchy, computed once outside the timed
    # region; the coarsening is deterministic, so partition sees the same levels
    h = J.coarsen(dg, k, seed=seed)
    lv_nnz = []
    for i in range(h.levels):
        view = J.Csr()
        mp = J.C.c_void_p()
        J.lib().jet_hierarchy_level(h.h, i, J.C.byref(view), J.C.byref(mp))
        lv_nnz.append(int(view.nnz))
    h.close()
    # warm-up calls are the timed call itself (same flags and trace buffer)
    for _ in range(warmup):
        J.partition(dg, k, seed=seed, flags=J.JET_F_PROFILE, trace_cap=1 << 16)
    torch.cuda.synchronize()
    # no Python garbage collection inside the timed region (a full collection
    # of the interpreter's heap costs tens of milliseconds)
    gc.collect()
    gc.disable()
    res = []
    t_ret = []
    t0 = time.perf_counter()
    for _ in range(steps):
        part, st, tr = J.partition(dg, k, seed=seed, flags=J.JET_F_PROFILE, trace_cap=1 << 16)
        res.append((st, tr))
        t_ret.append(time.perf_counter())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gc.enable()
    ms_per_step = (t1 - t0) * 1e3 / steps
    st0, tr0 = res[0]
    edges_per_step = sum(lv_nnz[r["level"]] for r in tr0)
    # roofline of the finest level's gain pass, over all timed steps
    ms_gain = sum(s["ms_gain"] for s, _ in res)
    passes = sum(s["gain_passes"] for s, _ in res)
    # finest level: one graph whose degrees all lie in [1, 32] has no class list
    deg = np.diff(g.xadj)
    listed = not (g.n > 0 and int(deg.min()) >= 1 and int(deg.max()) <= 32)
    # |X| of each finest-level Jetlp pass, from the trace (one record per iteration)
    gbytes = sum(gain_bytes(s["gain_entries"], s["gain_rows"], s["gain_vertices"], not w["unit"], listed,
                            compact=k <= 256,
                            in_x=sum(r["nX"] for r in tr if r["level"] == 0 and r["kind"] == 1))
                 for s, tr in res)
    achieved = (gbytes / passes) / ((ms_gain / passes) * 1e-3) / 1e9 if passes else 0.0
    refine_ms = sum(s["ms_refine"] for s, _ in res) / steps
    fin = [r for r in tr0 if r["level"] == 0]
    traffic, tdetail = measured_traffic(name)
    # second ceiling: one pass that only streams the CSR and gathers the
    # neighbours' parts (the floor of any pass over every entry)
    gms = J.gather_ceiling(dg, part, k, reps=10)
    pbytes = 1 if k <= 256 else 2
    gbytes_ceiling = g.nnz * (4 if w["unit"] else 8) + pbytes * g.n
    gather = {"ms": gms, "GBs": gbytes_ceiling / (gms * 1e-3) / 1e9,
              "kernel": f"k_gather_ceiling: every CSR entry (id, weight) read and its neighbour's {8 * pbytes}-bit "
                        f"part gathered, 16 entries per thread; algorithmic bytes 4 or 8 per entry + {pbytes} per "
                        f"vertex"}
    return {
        "part": part, "dg": dg, "value": edges_per_step / (ms_per_step * 1e-3), "ms_per_step": ms_per_step,
        "config": {
            "workload": f"{w['label']}: multilevel partition, k={k}, lambda=3%, n={g.n}, 2m={g.nnz}, "
                        f"{'unit weights' if w['unit'] else 'edge weights 1..16'}",
            "k": k, "lambda_ppm": 30000, "n": g.n, "nnz": g.nnz, "levels": st0["levels"],
            "iters": st0["iters"], "lp_iters": st0["lp_iters"], "rw_iters": st0["rw_iters"],
            "rs_iters": st0["rs_iters"], "finest_iters": len(fin), "cut": st0["cut"],
            "balanced": bool(st0["balanced"]), "ms_coarsen": st0["ms_coarsen"],
            "ms_refine": refine_ms,
            "ms_gpu_total": sum(s["ms_total"] for s, _ in res) / steps,
            "ms_wall_steps": [round((b - a) * 1e3, 2) for a, b in zip([t0] + t_ret[:-1], t_ret)],
            "refine_only_edges_per_s": edges_per_step / (refine_ms * 1e-3) if refine_ms else None,
            "edges_per_step": edges_per_step,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "connectivity/gain pass of the finest level's Jetlp iterations: every launch between "
                      "the HIP events around the pass (" + w["gain_kernels"] + ")",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_detail": tdetail,
            "copy_ceiling_GBs": ceiling["GBs"] if ceiling else None,
            "frac_of_copy_ceiling": achieved / ceiling["GBs"] if ceiling else None,
            "gather_ceiling": gather,
            "frac_of_gather_ceiling": achieved / gather["GBs"] if gather["GBs"] else None,
            "bytes_per_pass": gbytes / passes if passes else None,
            # the scope table's all-rows formula (every row's entries, 30 B per
            # vertex), beside the method's bytes above (locked rows skipped)
            "all_rows_formula_bytes": g.nnz * (4 if w["unit"] else 8) + 30 * g.n,
            "frac_all_rows_formula": ((g.nnz * (4 if w["unit"] else 8) + 30 * g.n) / ((ms_gain / passes) * 1e-3) / 1e9
                                      / HBM_PEAK_GBS) if passes else None,
            "ms_per_pass": ms_gain / passes if passes else None,
            "passes": passes,
        },
    }


def cpu_baseline_full(g, k, seed, gpu_part, gpu_cut, edges_of_level):
    """The oracle's whole multilevel partition of the same graph, one thread."""
    import numpy as np
    from oracle import oracle as O
    O.lib()
    t0 = time.perf_counter()
    res = O.partition(g, k, seed=seed, trace_cap=1 << 20)
    dt = time.perf_counter() - t0
    edges = sum(edges_of_level[r["level"]] for r in res["trace"]) if len(res["level_sizes"]) == len(
        edges_of_level) else 0
    return {
        "value": edges / dt if dt > 0 else None, "unit": "edges/s", "cores": 1, "kind": "oracle",
        "sample": f"the oracle's whole multilevel partition of the same graph (k={k}, seed={seed}), one "
                  f"thread, {len(res['trace'])} iterations over {len(res['level_sizes'])} levels, {dt:.1f} s; "
                  f"oracle cut {res['cut']} vs GPU cut {gpu_cut}",
        "seconds": dt,
        "identical_partition": bool(np.array_equal(res["part"], gpu_part)),
        **host_info(),
    }


def cpu_baseline_sample(J, g, dg, k, seed, iters):
    """The oracle's refinement of the finest level (level 0 parameters) from
    the seeded random partition, capped at `iters` iterations, one thread;
    the GPU runs the same refinement and must return the same partition."""
    import numpy as np
    import torch
    from oracle import oracle as O
    from paper_2304_13194_amd import inputs as I
    O.lib()
    p0 = I.random_partition(g.n, k, seed)
    t0 = time.perf_counter()
    res = O.refine(g, p0, k, seed=seed, max_iters=iters, trace_cap=iters + 1)
    dt = time.perf_counter() - t0
    gp = torch.from_numpy(p0.copy()).cuda()
    st, tr, _ = J.refine(dg, gp, k, seed=seed, max_iters=iters, trace_cap=iters + 1)
    torch.cuda.synchronize()
    same = bool(np.array_equal(gp.cpu().numpy(), res.part)) and tr == res.trace
    kinds = {1: "Jetlp", 2: "Jetrw", 3: "Jetrs"}
    return {
        "value": res.iters * g.nnz / dt if dt > 0 else None, "unit": "edges/s", "cores": 1, "kind": "oracle",
        "sample": f"the oracle's refinement of the finest level of the same graph (level-0 parameters, k={k}) "
                  f"from the seeded random partition, capped at {iters} iterations "
                  f"({', '.join(kinds[r['kind']] for r in res.trace)}), one thread, {dt:.1f} s: "
                  f"{res.iters} x 2m edges / time. Refinement only (no coarsening in its time), so it "
                  f"flatters the CPU against `value`; compare with config.refine_only_edges_per_s",
        "seconds": dt,
        "identical_partition": same,
        **host_info(),
    }


def batch_bench(J, graphs, spec, reps=2, oracle=True):
    """512 RGGs: one jet_refine_batch call vs one jet_refine per graph; the
    oracle's refinement of the same graphs on one core (a bounded sample)
    and on every core (all 512)."""
    import torch
    from paper_2304_13194_amd import inputs as I
    dgs = [J.to_device(g, unit_vwgt=True, unit_adjwgt=True) for g in graphs]
    p0 = [torch.from_numpy(I.random_partition(g.n, k, s)).cuda() for g, (n, k, s) in zip(graphs, spec)]
    params = [dict(k=k, seed=s) for (n, k, s) in spec]
    torch.cuda.synchronize()
    # batched: warm-up, then timed calls on fresh copies of P_0
    parts = [p.clone() for p in p0]
    J.refine_batch(dgs, parts, params)
    times = []
    for _ in range(reps):
        parts = [p.clone() for p in p0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats, _ = J.refine_batch(dgs, parts, params)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    t_batch = min(times)
    # one call per graph
    single = [p.clone() for p in p0]
    for dg, p, prm in zip(dgs[:8], [q.clone() for q in p0[:8]], params[:8]):
        J.refine(dg, p, **prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sstats = [J.refine(dg, p, **prm)[0] for dg, p, prm in zip(dgs, single, params)]
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    identical = all(torch.equal(a, b) for a, b in zip(parts, single))
    cut_b = sum(s["cut"] for s in stats)
    cut_s = sum(s["cut"] for s in sstats)
    edges = sum(s["iters"] * g.nnz for s, g in zip(stats, graphs))
    out = {
        "workload": f"{len(graphs)} RGGs (mean degree 10, n log-uniform in [1e3, 2e5], sum n = "
                    f"{sum(g.n for g in graphs)}, sum 2m = {sum(g.nnz for g in graphs)}), k in {{2..128}}, "
                    f"lambda 3%, seeded random P_0, single-level refinement",
        "graphs_per_s_batched": len(graphs) / t_batch,
        "graphs_per_s_one_per_launch": len(graphs) / t_single,
        "speedup": t_single / t_batch,
        "ms_batched": t_batch * 1e3,
        "ms_one_per_launch": t_single * 1e3,
        "refine_edges_per_s_batched": edges / t_batch,
        "iters_max": max(s["iters"] for s in stats),
        "iters_mean": sum(s["iters"] for s in stats) / len(stats),
        "total_cut": cut_b,
        "identical_partitions": bool(identical and cut_b == cut_s),
    }
    if oracle:
        out["oracle"] = batch_oracle(spec)
    return out


def batch_oracle(spec, budget_s=10.0):
    """The oracle on the batch's graphs. One core: graphs in a seeded order
    until about budget_s of refinement, scaled to graphs/s. All cores: every
    graph, dealt round robin to one worker per core; each worker times only
    its refinements, and the makespan is the slowest worker's sum."""
    import numpy as np
    from oracle import oracle as O
    from paper_2304_13194_amd import inputs as I
    O.lib()
    order = np.argsort(I.stream(4243, np.arange(len(spec), dtype=np.uint64)), kind="stable")
    t_one, done, n_one = 0.0, 0, 0
    for i in order:
        n, k, s = spec[int(i)]
        g = I.rgg(n, s)
        p0 = I.random_partition(g.n, k, s)
        t0 = time.perf_counter()
        O.refine(g, p0, k, seed=s)
        t_one += time.perf_counter() - t0
        done += 1
        n_one += n
        if t_one >= budget_s:
            break
    nw = pool_workers()
    chunks = [[spec[i] for i in range(w, len(spec), nw)] for w in range(nw)]
    import multiprocessing as mp
    with ProcessPoolExecutor(max_workers=nw, mp_context=mp.get_context("spawn"), initializer=_worker_init) as ex:
        per = list(ex.map(_oracle_refine_job, chunks))
    makespan = max(sum(p) for p in per)
    return {
        "one_core": {"graphs_per_s": done / t_one, "graphs": done, "seconds": t_one,
                     "sample": f"{done} of {len(spec)} graphs in a seeded order (sum n = {n_one}), one thread"},
        "all_cores": {"graphs_per_s": len(spec) / makespan, "graphs": len(spec), "seconds": makespan,
                      "workers": nw,
                      "sample": "every graph, dealt round robin to one worker process per core; each worker "
                                "times its own refinements (generation excluded); seconds = slowest worker"},
        **host_info(),
    }


def serve_bench(J, jobs, graphs, budget_bytes, warmup, rates=(50, 100, 200, 500, 1000, 2000), slots=256):
    """Poisson arrivals into jet_server vs the same jobs one at a time. Every
    job is drawn on its own (grid side, or R-MAT scale, edge factor and graph
    seed; k; seed); the first `warmup` jobs of each rate are not measured."""
    import numpy as np
    import torch
    from paper_2304_13194_amd import inputs as I
    dgs = [J.to_device(g, unit_vwgt=(sp[0] == "grid"), unit_adjwgt=(sp[0] == "grid"))
           for g, (sp, _, _) in zip(graphs, jobs)]
    # one at a time (jet_partition): reference results and sequential throughput
    for dg, (_, k, seed) in list(zip(dgs, jobs))[:4]:
        J.partition(dg, k, seed=seed)
    torch.cuda.synchronize()
    ref = []
    t0 = time.perf_counter()
    for dg, (_, k, seed) in zip(dgs, jobs):
        part, st, _ = J.partition(dg, k, seed=seed)
        ref.append((part, st["cut"]))
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    nmeas = len(jobs) - warmup
    # one long-lived server for every rate, warmed by the first rate's
    # unmeasured jobs (its lanes' workspaces and memory pools then hold what
    # the mix needs, as the one-at-a-time context's do)
    sv = J.Server(hbm_budget_bytes=budget_bytes, max_slots=slots)
    out = {"workload": f"{nmeas} measured + {warmup} warm-up jobs per rate, each drawn on its own: half 2-D "
                       f"grids (side uniform in [64, 1024]), half R-MAT graphs (scale uniform in [12, 20], edge "
                       f"factor uniform in [8, 16], weights 1..16); k uniform in [2, 256], lambda 3%",
           "hbm_budget_bytes": budget_bytes, "max_slots": slots,
           "graphs_per_s_one_at_a_time": len(jobs) / t_seq, "rates": []}
    identical = True
    steps0 = jobs0 = 0
    try:
        for ri, rate in enumerate(rates):
            arr = I.arrivals(rate, len(jobs), 500 + ri)
            outs = [torch.empty(dg.n, dtype=torch.int32, device="cuda") for dg in dgs]
            torch.cuda.synchronize()
            peak_inuse, held = 0, 0
            tickets = []
            t0 = time.perf_counter()
            for dg, (_, k, seed), at, o in zip(dgs, jobs, arr, outs):
                d = t0 + at - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                tickets.append(sv.submit(dg, o, k, seed=seed))
                inf = sv.info()
                peak_inuse = max(peak_inuse, inf["hbm_in_use"])
                held = max(held, inf["queued"])
            res = [sv.wait(t, 600000) for t in tickets]
            info = sv.info()
            steps, sjobs = info["steps"] - steps0, info["step_jobs"] - jobs0
            steps0, jobs0 = info["steps"], info["step_jobs"]
            m = res[warmup:]
            out["rates"].append(_rate_row(rate, m, res, outs, ref, peak_inuse, held, steps, sjobs))
            identical = identical and out["rates"][-1].pop("_ok")
    finally:
        sv.close()
    out["identical_to_alone"] = bool(identical)
    return out


def _rate_row(rate, m, res, outs, ref, peak_inuse, held, steps, sjobs):
    """Latency and throughput of the measured jobs `m` of one arrival rate;
    _ok: every job (warm-up included) equals its one-at-a-time result."""
    import numpy as np
    import torch
    lat = np.array([r["t_done_ms"] - r["t_submit_ms"] for r in m])
    qwait = np.array([r["t_admit_ms"] - r["t_submit_ms"] for r in m])
    span = (max(r["t_done_ms"] for r in m) - min(r["t_submit_ms"] for r in m)) * 1e-3
    ok = all(r["status"] == 0 and r["cut"] == c and torch.equal(o, p) for r, o, (p, c) in zip(res, outs, ref))
    return {"rate_jobs_per_s": rate, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "graphs_per_s": len(m) / span,
            "p50_admission_wait_ms": float(np.percentile(qwait, 50)),
            "max_queued_seen": held, "max_hbm_in_use_seen": peak_inuse,
            "mean_jobs_per_step": sjobs / max(steps, 1), "steps": steps, "_ok": ok}


def ablation_bench(J, dg, k, seed, label):
    """Jetlp ablations and the phi sweep (Section 7.1, Component Effectiveness, Table lp_versions) on one
    graph: cut and time of the full multilevel partition per variant."""
    import torch
    NL, NA = J.JET_F_LP_NO_LOCKS, J.JET_F_LP_NO_AFTERBURNER
    variants = [("baseline sync LP", dict(c=(0, 1), flags=NL | NA)),
                ("+locks", dict(c=(0, 1), flags=NA)),
                ("+weak afterburner", dict(c=(0, 1), flags=NL)),
                ("+full afterburner", dict(flags=NL)),
                ("full Jetlp", dict()),
                ("full Jetlp, phi 0.99", dict(phi=(99, 100))),
                ("full Jetlp, phi 0.9999", dict(phi=(9999, 10000))),
                ("full Jetlp, two-hop coarsening", dict(flags=J.JET_F_TWO_HOP)),
                ("full Jetlp, graph-growing start", dict(flags=J.JET_F_BFS_START)),
                ("full Jetlp, persistent connectivity table (Section 4.3, Algorithm 6)",
                 dict(flags=J.JET_F_CONN_TABLE))]
    rows = []
    for name, kw in variants:
        J.partition(dg, k, seed=seed, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        part, st, _ = J.partition(dg, k, seed=seed, **kw)
        torch.cuda.synchronize()
        rows.append({"variant": name, "cut": st["cut"], "balanced": bool(st["balanced"]),
                     "ms": round((time.perf_counter() - t0) * 1e3, 2), "ms_refine": round(st["ms_refine"], 2),
                     "iters": st["iters"]})
    return {"graph": label, "k": k, "rows": rows}


def level_edges(J, dg, k, seed):
    """2m of every hierarchy level (the coarsening is deterministic)."""
    h = J.coarsen(dg, k, seed=seed)
    out = []
    for i in range(h.levels):
        view = J.Csr()
        mp = J.C.c_void_p()
        J.lib().jet_hierarchy_level(h.h, i, J.C.byref(view), J.C.byref(mp))
        out.append(int(view.nnz))
    h.close()
    return out


def say(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat22", choices=sorted(WORKLOADS))
    ap.add_argument("--secondary", default="stencil128", choices=sorted(WORKLOADS) + ["none"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-ablations", action="store_true")
    ap.add_argument("--no-copy-ceiling", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=8,
                    help="iterations of the oracle's sampled refinement (R-MAT workload)")
    ap.add_argument("--serve-jobs", type=int, default=200, help="measured jobs per arrival rate")
    ap.add_argument("--serve-warmup", type=int, default=20, help="unmeasured jobs before them")
    ap.add_argument("--serve-budget-gb", type=float, default=16.0, help="server HBM budget (GB)")
    ap.add_argument("--serve-slots", type=int, default=256, help="server slots (jobs admitted at once)")
    ap.add_argument("--serve-rates", default="50,100,200,500,1000,2000", help="arrival rates (jobs/s)")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--graph-cache", default=None,
                    help="directory: reuse generated main graphs across runs (.npz, no pickle)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a plain 256 MiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the refinement of one graph "
              "runs on a single MI355X); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2304_13194_amd import inputs as I
    from paper_2304_13194_amd import jet as J

    if args.calib_copy:
        # known traffic: the copy reads and writes 2^28 bytes each
        src = torch.ones(1 << 26, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # inputs of the batch and serving runs are generated in worker processes
    # once the partition timings and the CPU baselines are done: generation
    # running beside a timed partition slows the host thread that drives it
    pool_ex = None
    fut_rgg = fut_srv = None
    spec = None
    jobs = I.serve_job_specs(args.serve_jobs + args.serve_warmup)
    ceiling = None if args.no_copy_ceiling else copy_ceiling()
    if ceiling:
        say(f"copy ceiling {ceiling['GBs']:.0f} GB/s")

    def run(name):
        w = WORKLOADS[name]
        t = time.perf_counter()
        say(f"generating {name}")
        g = load_or_make_graph(w, name, args.graph_cache)
        t = time.perf_counter() - t
        say(f"{name}: n={g.n} 2m={g.nnz} in {t:.1f} s; timing {args.steps} partitions")
        m = measure_workload(J, name, g, w, args.seed, args.steps, args.warmup, ceiling)
        m["config"]["gen_s"] = t
        say(f"{name}: {m['ms_per_step']:.1f} ms per partition, gain pass {m['roofline']['frac'] * 100:.1f}% of HBM")
        return g, m

    g, main_m = run(args.workload)
    w = WORKLOADS[args.workload]
    out = {
        "metric": "Jet refine edges/s per iteration (sum over refinement iterations of the level's 2m, "
                  "per second of full partition time)",
        "value": main_m["value"],
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32/int64",
        "data": "synthetic",
        "config": main_m["config"],
        "roofline": main_m["roofline"],
        "copy_ceiling": ceiling,
    }
    if not args.no_cpu_baseline and int(os.environ.get("RANK", "0")) == 0:
        say("cpu baseline (oracle)")
        part = main_m["part"].cpu().numpy()
        if w["kind"] == "rmat":
            out["cpu_baseline"] = cpu_baseline_sample(J, g, main_m["dg"], w["k"], args.seed, args.cpu_iters)
        else:
            out["cpu_baseline"] = cpu_baseline_full(g, w["k"], args.seed, part, main_m["config"]["cut"],
                                                    level_edges(J, main_m["dg"], w["k"], args.seed))
    if not args.no_ablations:
        say("ablations")
        out["ablations"] = [ablation_bench(J, main_m["dg"], w["k"], args.seed, f"{w['label']} (n={g.n})")]
    del main_m["dg"], main_m["part"]
    del g
    gc.collect()
    torch.cuda.empty_cache()
    if args.secondary != "none" and args.secondary != args.workload:
        g2, sec = run(args.secondary)
        w2 = WORKLOADS[args.secondary]
        s_out = {"value": sec["value"], "unit": "edges/s", "ms_per_step": sec["ms_per_step"],
                 "config": sec["config"], "roofline": sec["roofline"]}
        if not args.no_cpu_baseline:
            say("secondary cpu baseline (oracle)")
            if w2["kind"] == "rmat":
                s_out["cpu_baseline"] = cpu_baseline_sample(J, g2, sec["dg"], w2["k"], args.seed, args.cpu_iters)
            else:
                s_out["cpu_baseline"] = cpu_baseline_full(g2, w2["k"], args.seed, sec["part"].cpu().numpy(),
                                                          sec["config"]["cut"],
                                                          level_edges(J, sec["dg"], w2["k"], args.seed))
        if not args.no_ablations:
            out["ablations"].append(ablation_bench(J, sec["dg"], w2["k"], args.seed, f"{w2['label']} (n={g2.n})"))
        out["secondary"] = s_out
        del sec, g2
        gc.collect()
        torch.cuda.empty_cache()
    if not (args.no_batch and args.no_serve):
        import multiprocessing as mp
        say("generating batch and serving inputs")
        pool_ex = ProcessPoolExecutor(max_workers=max(1, pool_workers() - 2), mp_context=mp.get_context("spawn"),
                                      initializer=_worker_init)
        if not args.no_batch:
            spec = I.rgg_batch_spec()
            fut_rgg = [pool_ex.submit(_gen_rgg, (n, s)) for n, _, s in spec]
        if not args.no_serve:
            fut_srv = [pool_ex.submit(_gen_pool_graph, sp) for sp, _, _ in jobs]
        # every input is ready before the first timed batch or serving run
        for f in (fut_rgg or []) + (fut_srv or []):
            f.exception()
    if fut_rgg is not None:
        say("batch")
        try:
            graphs = [f.result() for f in fut_rgg]
            out["batch"] = batch_bench(J, graphs, spec, oracle=not args.no_cpu_baseline)
            del graphs
        except Exception as e:  # reported, never hidden
            out["batch"] = {"error": repr(e)}
        gc.collect()
        torch.cuda.empty_cache()
    if fut_srv is not None:
        say("serving")
        try:
            graphs = [f.result() for f in fut_srv]
            out["serving"] = serve_bench(J, jobs, graphs, int(args.serve_budget_gb * 1e9), args.serve_warmup,
                                         rates=tuple(float(x) for x in args.serve_rates.split(",")),
                                         slots=args.serve_slots)
            del graphs
        except Exception as e:
            out["serving"] = {"error": repr(e)}
    if pool_ex is not None:
        pool_ex.shutdown()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
