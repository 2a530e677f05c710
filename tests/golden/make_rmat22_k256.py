"""Writes rmat22_k256.json: the oracle's multilevel partition of the R-MAT
scale-22 graph (edge factor 16, (a,b,c,d) = (0.57,0.19,0.19,0.05), edge
weights 1..16, generator master seed 3), k = 256, lambda 3%, seed 2.

Calls only the oracle (Algorithm 1 with Algorithms 3-5 and Jetrs on every
level) and the seeded input generator. Stored: every per-iteration trace
record of every level, the level sizes, the SHA-256 of the graph's CSR arrays, the final cut / largest part weight /
balance, the SHA-256 of the final partition (int32, little endian) and the
parts of 4096 sampled vertices, so that a mismatch can be located.

    python tests/golden/make_rmat22_k256.py      (about ten minutes, one core)
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

SCALE, EF, GEN_SEED, K, SEED = 22, 16, 3, 256, 2
SAMPLE = 4096


def sample_ids(n, count=SAMPLE):
    """Evenly spread vertex ids plus the last one (covers the ragged end)."""
    ids = np.unique(np.concatenate([np.linspace(0, n - 1, count - 1).astype(np.int64), [n - 1]]))
    return ids


def graph_sha256(g):
    """SHA-256 over the CSR arrays (xadj int64, adjncy, vwgt, adjwgt int32; little endian)."""
    h = hashlib.sha256()
    for arr, dt in ((g.xadj, "<i8"), (g.adjncy, "<i4"), (g.vwgt, "<i4"), (g.adjwgt, "<i4")):
        h.update(np.ascontiguousarray(arr, dtype=dt).tobytes())
    return h.hexdigest()


def main():
    from oracle import oracle as O
    from paper_2304_13194_amd import inputs as I
    t0 = time.perf_counter()
    g = I.rmat(SCALE, EF, GEN_SEED)
    print(f"R-MAT scale {SCALE}: n={g.n} 2m={g.nnz} in {time.perf_counter() - t0:.1f} s", flush=True)
    t0 = time.perf_counter()
    res = O.partition(g, K, seed=SEED, trace_cap=1 << 20)
    dt = time.perf_counter() - t0
    part = np.ascontiguousarray(res["part"], dtype="<i4")
    ids = sample_ids(g.n)
    out = {
        "source": "oracle/jet_oracle.c og_partition (Algorithm 1; Algorithms 3, 4, 5 and Jetrs per level)",
        "graph": {"kind": "rmat", "scale": SCALE, "edge_factor": EF, "gen_seed": GEN_SEED,
                  "n": int(g.n), "nnz": int(g.nnz), "sha256": graph_sha256(g)},
        "k": K, "seed": SEED, "lambda_ppm": 30000,
        "level_sizes": [int(x) for x in res["level_sizes"]],
        "cut": res["cut"], "maxw": res["maxw"], "balanced": res["balanced"], "o": res["o"],
        "part_sha256": hashlib.sha256(part.tobytes()).hexdigest(),
        "sample_ids": [int(x) for x in ids],
        "sample_parts": [int(x) for x in part[ids]],
        "trace": res["trace"],
        "oracle_seconds": round(dt, 1),
    }
    path = os.path.join(HERE, "rmat22_k256.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(f"{len(res['trace'])} iterations over {len(res['level_sizes'])} levels, cut {res['cut']}, "
          f"{dt:.1f} s -> {path}", flush=True)


if __name__ == "__main__":
    main()
