"""Benchmark: Jet refinement throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload stencil128|rmat22|grid64]

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
  cpu_baseline the CPU oracle (single thread, this host), same unit, on a
               bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # configs[1]: full multilevel partition of the 128^3 27-point mesh, k = 64
    "stencil128": dict(kind="stencil", side=128, k=64, unit=True),
    # configs[2]: R-MAT scale 22, edge factor 16, weights in [1, 16], k = 256
    "rmat22": dict(kind="rmat", scale=22, ef=16, k=256, unit=False),
    # configs[0]: 64 x 64 grid, k = 4 (single level in the config; here multilevel)
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


def gain_bytes(entries, rows, vertices, weighted):
    """Algorithmic bytes of a connectivity/gain pass.

    Per CSR entry of an unlocked row: 4 B neighbour id (+4 B edge weight when
    weights are passed). Per unlocked row: 8 B row offsets, 4 B for its part
    id gathered by neighbours (counted once). Per visited vertex: 4 B list
    entry, 4 B own part, 4 B lock stamp, 8 B record written.
    """
    return entries * (8 if weighted else 4) + rows * 12 + vertices * 20


def cpu_baseline(g, k, seed, budget_s=25.0):
    """The oracle's multilevel partition of the same graph, single thread."""
    from oracle import oracle as O
    O.lib()
    t0 = time.perf_counter()
    res = O.partition(g, k, seed=seed, trace_cap=1 << 20)
    dt = time.perf_counter() - t0
    sizes = res["level_sizes"]
    return res, dt, sizes


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="stencil128", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=2)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (the refinement of one graph "
              "runs on a single MI355X); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2304_13194_amd import jet as J

    w = WORKLOADS[args.workload]
    k = w["k"]
    t_gen = time.perf_counter()
    g = make_graph(w)
    t_gen = time.perf_counter() - t_gen
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

    for _ in range(args.warmup):
        J.partition(dg, k, seed=args.seed)
    torch.cuda.synchronize()

    steps = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        part, st, tr = J.partition(dg, k, seed=args.seed, flags=J.JET_F_PROFILE, trace_cap=1 << 16)
        steps.append((st, tr))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    st0, tr0 = steps[0]
    edges_per_step = sum(lv_nnz[r["level"]] for r in tr0)
    value = edges_per_step / (ms_per_step * 1e-3)
    # roofline of the finest level's gain pass, over all timed steps
    ms_gain = sum(s["ms_gain"] for s, _ in steps)
    passes = sum(s["gain_passes"] for s, _ in steps)
    gbytes = sum(gain_bytes(s["gain_entries"], s["gain_rows"], s["gain_vertices"], not w["unit"])
                 for s, _ in steps)
    achieved = (gbytes / passes) / ((ms_gain / passes) * 1e-3) / 1e9 if passes else 0.0
    refine_ms = sum(s["ms_refine"] for s, _ in steps) / args.steps
    fin = [r for r in tr0 if r["level"] == 0]

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
            "refine_only_edges_per_s": edges_per_step / (refine_ms * 1e-3) if refine_ms else None,
            "gen_s": t_gen,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_gain (connectivity/gain pass, finest level, Jetlp iterations)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "bytes_per_pass": gbytes / passes if passes else None,
            "ms_per_pass": ms_gain / passes if passes else None,
            "passes": passes,
        },
    }
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
