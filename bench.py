"""Benchmark: Jet refinement on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload stencil128|rmat22|grid64]
                    [--no-cpu-baseline] [--no-batch] [--no-serve] [--no-ablations]

A step is one full multilevel partition (Algorithm 1: heavy-edge coarsening,
seeded random coarsest partition, Jet refinement of every level, i.e. every
row of the refinement hot path) of a device-resident synthetic graph. The
default workload is the 128^3 27-point stencil mesh (2,097,152 vertices,
53,645,816 CSR entries, unit weights), k = 64, lambda = 3%.

Prints one JSON line:
  value        edges traversed by Jet iterations per second of step time:
               sum over the refinement iterations of all levels of that
               level's CSR entries (2m), divided by the whole step's wall
               time (coarsening and set-up included)
  roofline     the connectivity/gain pass of the finest level's Jetlp
               iterations: algorithmic bytes per pass / average pass time
               (HIP events around each pass, on the library's stream),
               against 8 TB/s HBM
  cpu_baseline the CPU oracle (single thread, this host), same unit, on the
               same workload
  batch        512 random geometric graphs refined in one jet_refine_batch
               call vs one jet_refine call per graph (graphs/s, identical
               partitions required)
  serving      Poisson arrivals of partition jobs (grids and R-MAT graphs)
               into jet_server: p50 / p99 latency and graphs/s per arrival
               rate, vs partitioning the same jobs one at a time
  ablations    Jetlp variants (baseline synchronous LP, +locks, +weak or
               full afterburner, full Jetlp), phi 0.99 / 0.999 / 0.9999 and
               two-hop coarsening on the main graph and the serving pool's
               largest R-MAT graph: cut and partition time per variant
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
# the kernel source they were taken on (profiles/k_gain_stencil128_k64.md).
TRAFFIC = {
    "stencil128": dict(src_sha256="033629e58bb3ac3b35fbce81e7ab0b8ab8de40d2e94523d1bab68f49dcbc511b",
                       fetch=249198497, write=17431882, fetch_factor=1.9997, write_factor=1.0),
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
    # full multilevel partition of the 128^3 27-point mesh, k = 64
    "stencil128": dict(kind="stencil", side=128, k=64, unit=True),
    # R-MAT scale 22, edge factor 16, weights in [1, 16], k = 256
    "rmat22": dict(kind="rmat", scale=22, ef=16, k=256, unit=False),
    # 64 x 64 grid, k = 4
    "grid64": dict(kind="grid", side=64, k=4, unit=True),
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


def gain_bytes(entries, rows, vertices, weighted, listed=True):
    """Algorithmic bytes of a connectivity/gain pass.

    Per CSR entry of an unlocked row: 4 B neighbour id (+4 B edge weight when
    weights are passed). Per unlocked row: 8 B row offsets, 4 B for its part
    id gathered by neighbours (counted once). Per visited vertex: 4 B list
    entry (none when every vertex is in the small-row class, whose list is
    then the identity and is not read), 4 B own part, 4 B lock stamp, 8 B
    record written.
    """
    return entries * (8 if weighted else 4) + rows * 12 + vertices * (20 if listed else 16)


# ------------------------------------------------------------ input makers --
# (module-level so a process pool can run them)

def _gen_rgg(args):
    from paper_2304_13194_amd import inputs as I
    n, seed = args
    return I.rgg(n, seed)


def _gen_pool_graph(spec):
    from paper_2304_13194_amd import inputs as I
    return I.serve_pool_graph(spec)


# -------------------------------------------------------------- sub-benches --

def batch_bench(J, graphs, spec, reps=2):
    """512 RGGs: one jet_refine_batch call vs one jet_refine per graph."""
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
    return {
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


def serve_bench(J, pool, jobs, rates=(50, 200, 1000, 2000)):
    """Poisson arrivals into jet_server vs the same jobs one at a time."""
    import numpy as np
    import torch
    from paper_2304_13194_amd import inputs as I
    dgs = [J.to_device(g, unit_vwgt=(s[0] == "grid"), unit_adjwgt=(s[0] == "grid")) for g, s in zip(pool, I.SERVE_POOL)]
    # one at a time (jet_partition): reference results and sequential throughput
    for gi, k, seed in jobs[:4]:
        J.partition(dgs[gi], k, seed=seed)
    torch.cuda.synchronize()
    ref = []
    t0 = time.perf_counter()
    for gi, k, seed in jobs:
        part, st, _ = J.partition(dgs[gi], k, seed=seed)
        ref.append((part, st["cut"]))
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    out = {"workload": f"{len(jobs)} jobs per rate drawn from grids (side 64..1024) and R-MAT graphs "
                       f"(scale 12..20, edge factor 8/16, weights 1..16), k uniform in [2, 256], lambda 3%",
           "graphs_per_s_one_at_a_time": len(jobs) / t_seq, "rates": []}
    identical = True
    for ri, rate in enumerate(rates):
        arr = I.arrivals(rate, len(jobs), 500 + ri)
        outs = [torch.empty(dgs[gi].n, dtype=torch.int32, device="cuda") for gi, _, _ in jobs]
        torch.cuda.synchronize()
        sv = J.Server(hbm_budget_bytes=128 << 30, max_slots=64)
        try:
            tickets = []
            t0 = time.perf_counter()
            for (gi, k, seed), at, o in zip(jobs, arr, outs):
                d = t0 + at - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                tickets.append(sv.submit(dgs[gi], o, k, seed=seed))
            res = [sv.wait(t, 600000) for t in tickets]
            info = sv.info()
        finally:
            sv.close()
        lat = np.array([r["t_done_ms"] - r["t_submit_ms"] for r in res])
        span = (max(r["t_done_ms"] for r in res) - min(r["t_submit_ms"] for r in res)) * 1e-3
        ok = all(r["status"] == 0 and r["cut"] == c and torch.equal(o, p)
                 for r, o, (p, c) in zip(res, outs, ref))
        identical = identical and ok
        out["rates"].append({"rate_jobs_per_s": rate, "p50_ms": float(np.percentile(lat, 50)),
                             "p99_ms": float(np.percentile(lat, 99)), "graphs_per_s": len(jobs) / span,
                             "mean_jobs_per_step": info["step_jobs"] / max(info["steps"], 1),
                             "steps": info["steps"]})
    out["identical_to_alone"] = bool(identical)
    return out


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
                ("full Jetlp, graph-growing start", dict(flags=J.JET_F_BFS_START))]
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


def cpu_baseline(g, k, seed):
    """The oracle's multilevel partition of the same graph, single thread."""
    from oracle import oracle as O
    O.lib()
    t0 = time.perf_counter()
    res = O.partition(g, k, seed=seed, trace_cap=1 << 20)
    dt = time.perf_counter() - t0
    return res, dt, res["level_sizes"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="stencil128", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-ablations", action="store_true")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--graph-cache", default=None,
                    help="directory: reuse the generated main graph across runs (.npz, no pickle)")
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

    w = WORKLOADS[args.workload]
    k = w["k"]
    if args.calib_copy:
        # known traffic: the copy reads and writes 2^28 bytes each
        src = torch.ones(1 << 26, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # inputs of the batch and serving runs are generated in worker processes
    # while the main workload runs (none of it inside a timed region)
    pool_ex = None
    fut_rgg = fut_pool = None
    spec = serve = None
    if not (args.no_batch and args.no_serve):
        pool_ex = ProcessPoolExecutor(max_workers=6)
        if not args.no_batch:
            spec = I.rgg_batch_spec()
            fut_rgg = [pool_ex.submit(_gen_rgg, (n, s)) for n, _, s in spec]
        if not args.no_serve:
            fut_pool = [pool_ex.submit(_gen_pool_graph, s) for s in I.SERVE_POOL]
    t_gen = time.perf_counter()
    print(f"[bench] generating {args.workload}", file=sys.stderr, flush=True)
    g = load_or_make_graph(w, args.workload, args.graph_cache)
    t_gen = time.perf_counter() - t_gen
    print(f"[bench] graph n={g.n} 2m={g.nnz} in {t_gen:.1f} s", file=sys.stderr, flush=True)
    dg = J.to_device(g, unit_vwgt=w["unit"], unit_adjwgt=w["unit"])
    torch.cuda.synchronize()

    # level sizes (n, 2m) of the hierarchy, computed once outside the timed
    # region; the coarsening is deterministic, so partition sees the same levels
    h = J.coarsen(dg, k, seed=args.seed)
    lv_nnz = []
    for i in range(h.levels):
        view = J.Csr()
        mp = J.C.c_void_p()
        J.lib().jet_hierarchy_level(h.h, i, J.C.byref(view), J.C.byref(mp))
        lv_nnz.append(int(view.nnz))
    h.close()

    # warm-up calls are the timed call itself (same flags and trace buffer)
    for _ in range(args.warmup):
        J.partition(dg, k, seed=args.seed, flags=J.JET_F_PROFILE, trace_cap=1 << 16)
    torch.cuda.synchronize()

    # no Python garbage collection inside the timed region (a full collection
    # of the interpreter's heap costs tens of milliseconds)
    gc.collect()
    gc.disable()
    steps = []
    t_ret = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        part, st, tr = J.partition(dg, k, seed=args.seed, flags=J.JET_F_PROFILE, trace_cap=1 << 16)
        steps.append((st, tr))
        t_ret.append(time.perf_counter())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gc.enable()
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    st0, tr0 = steps[0]
    edges_per_step = sum(lv_nnz[r["level"]] for r in tr0)
    value = edges_per_step / (ms_per_step * 1e-3)
    # roofline of the finest level's gain pass, over all timed steps
    ms_gain = sum(s["ms_gain"] for s, _ in steps)
    passes = sum(s["gain_passes"] for s, _ in steps)
    # finest level: one graph whose degrees all lie in [1, 32] has no class list
    deg = np.diff(g.xadj)
    listed = not (g.n > 0 and int(deg.min()) >= 1 and int(deg.max()) <= 32)
    gbytes = sum(gain_bytes(s["gain_entries"], s["gain_rows"], s["gain_vertices"], not w["unit"], listed)
                 for s, _ in steps)
    achieved = (gbytes / passes) / ((ms_gain / passes) * 1e-3) / 1e9 if passes else 0.0
    refine_ms = sum(s["ms_refine"] for s, _ in steps) / args.steps
    fin = [r for r in tr0 if r["level"] == 0]
    traffic, tdetail = measured_traffic(args.workload)

    out = {
        "metric": "Jet refine edges/s per iteration (sum over refinement iterations of the level's 2m, "
                  "per second of full partition time)",
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32/int64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: multilevel partition, k={k}, lambda=3%, n={g.n}, 2m={g.nnz}, "
                        f"{'unit weights' if w['unit'] else 'weights 1..16'}",
            "k": k, "lambda_ppm": 30000, "n": g.n, "nnz": g.nnz, "levels": st0["levels"],
            "iters": st0["iters"], "lp_iters": st0["lp_iters"], "rw_iters": st0["rw_iters"],
            "rs_iters": st0["rs_iters"], "finest_iters": len(fin), "cut": st0["cut"],
            "balanced": bool(st0["balanced"]), "ms_coarsen": st0["ms_coarsen"],
            "ms_refine": refine_ms,
            "ms_gpu_total": sum(s["ms_total"] for s, _ in steps) / args.steps,
            "ms_wall_steps": [round((b - a) * 1e3, 2) for a, b in zip([t0] + t_ret[:-1], t_ret)],
            "refine_only_edges_per_s": edges_per_step / (refine_ms * 1e-3) if refine_ms else None,
            "gen_s": t_gen,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_gain<false, 1, 4, 8, 1> in Jetlp iterations (connectivity/gain pass of the small rows, finest level)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_detail": tdetail,
            "bytes_per_pass": gbytes / passes if passes else None,
            "ms_per_pass": ms_gain / passes if passes else None,
            "passes": passes,
        },
    }
    if not args.no_ablations:
        out["ablations"] = [ablation_bench(J, dg, k, args.seed, f"{args.workload} (n={g.n})")]
    if fut_rgg is not None:
        try:
            graphs = [f.result() for f in fut_rgg]
            out["batch"] = batch_bench(J, graphs, spec)
            del graphs
        except Exception as e:  # reported, never hidden
            out["batch"] = {"error": repr(e)}
    if fut_pool is not None:
        try:
            pool = [f.result() for f in fut_pool]
            out["serving"] = serve_bench(J, pool, I.serve_jobs(40))
            if not args.no_ablations:
                spec = I.SERVE_POOL[-1]  # the largest R-MAT of the pool
                dgr = J.to_device(pool[-1])
                out.setdefault("ablations", []).append(
                    ablation_bench(J, dgr, 64, args.seed, f"R-MAT scale {spec[1]}, edge factor {spec[2]} (n={pool[-1].n})"))
        except Exception as e:
            out["serving"] = {"error": repr(e)}
    if pool_ex is not None:
        pool_ex.shutdown()
    if not args.no_cpu_baseline and int(os.environ.get("RANK", "0")) == 0:
        res, dt, sizes = cpu_baseline(g, k, args.seed)
        # the oracle coarsens with the same rule, so its levels have the same sizes
        edges = 0
        if len(sizes) == len(lv_nnz):
            edges = sum(lv_nnz[r["level"]] for r in res["trace"])
        out["cpu_baseline"] = {
            "value": edges / dt if dt > 0 else None,
            "unit": "edges/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"oracle multilevel partition of the same graph (k={k}, seed={args.seed}), single "
                      f"thread, {len(res['trace'])} iterations over {len(sizes)} levels, {dt:.1f} s; "
                      f"oracle cut {res['cut']} vs GPU cut {st0['cut']}",
            "seconds": dt,
            "identical_partition": bool(np.array_equal(res["part"], part.cpu().numpy())),
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
