"""Seeded synthetic inputs: graphs in CSR form and initial partitions.

This module holds no refinement arithmetic. It only draws graphs and
partitions that both the device library and the CPU oracle consume.

All randomness comes from SplitMix64 (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014):

    mix64(z):  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9
               z ^= z >> 27; z *= 0x94D049BB133111EB
               z ^= z >> 31
    stream(seed, i) = mix64(seed + (i + 1) * 0x9E3779B97F4A7C15)   (mod 2**64)
    uniform integer in [0, r) = floor(x * r / 2**64) for x = stream(seed, i)

Graphs follow the problem statement of Section 2.1 of the paper: undirected,
no self-loops, no parallel edges, positive integer vertex and edge weights.
CSR arrays are ``xadj`` int64[n+1], ``adjncy`` int32[2m], ``vwgt`` int32[n],
``adjwgt`` int32[2m]; every undirected edge appears in both rows.

Sub-seed tags (``subseed(master, tag)``): 1 initial partition, 2 R-MAT bits,
3 edge weights, 4 vertex permutation, 5/6 RGG x/y, 7 RGG n, 8 k draw,
9 arrivals, 10 job mix.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def mix64_scalar(z: int) -> int:
    z &= (1 << 64) - 1
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & ((1 << 64) - 1)
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & ((1 << 64) - 1)
    z ^= z >> 31
    return z


def mix64(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def stream(seed: int, idx: np.ndarray) -> np.ndarray:
    """i-th SplitMix64 output of ``seed`` for every i in ``idx``."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & ((1 << 64) - 1)) + (idx + np.uint64(1)) * GAMMA
    return mix64(z)


def subseed(master: int, tag: int) -> int:
    return mix64_scalar((master ^ tag) & ((1 << 64) - 1))


def uniform_below(x: np.ndarray, r: int) -> np.ndarray:
    """floor(x * r / 2**64) for uint64 x and 1 <= r < 2**32, exactly."""
    assert 1 <= r < (1 << 32)
    x = np.asarray(x, dtype=np.uint64)
    rr = np.uint64(r)
    hi = x >> np.uint64(32)
    lo = x & np.uint64(0xFFFFFFFF)
    with np.errstate(over="ignore"):
        # hi*r + (lo*r >> 32) < 2**64 for r < 2**32, so nothing wraps.
        t = hi * rr + ((lo * rr) >> np.uint64(32))
    return (t >> np.uint64(32)).astype(np.int64)


@dataclass
class Graph:
    """CSR graph (host numpy arrays). ``vwgt``/``adjwgt`` are always explicit."""

    xadj: np.ndarray
    adjncy: np.ndarray
    vwgt: np.ndarray
    adjwgt: np.ndarray
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.xadj.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.xadj[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.xadj)


def _argsort_unique(key: np.ndarray) -> np.ndarray:
    """Ascending order of distinct int64 keys (any sort gives the same order
    when no two keys are equal). Large arrays use torch's multithreaded CPU
    sort; the order is identical to numpy's."""
    if key.shape[0] < (1 << 20):
        return np.argsort(key, kind="stable")
    import torch
    _, idx = torch.sort(torch.from_numpy(key), stable=True)
    return idx.numpy()


def csr_from_edges(n: int, u: np.ndarray, v: np.ndarray, w: np.ndarray | None = None,
                   vwgt: np.ndarray | None = None, name: str = "") -> Graph:
    """Symmetric CSR from a list of distinct undirected edges u < v (no self-loops).

    Rows are sorted by neighbour id.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    if w is None:
        w = np.ones(u.shape[0], dtype=np.int32)
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    ww = np.concatenate([w, w]).astype(np.int32)
    key = src * np.int64(n) + dst
    order = _argsort_unique(key)
    src = src[order]
    dst = dst[order]
    ww = ww[order]
    counts = np.bincount(src, minlength=n).astype(np.int64)
    xadj = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=xadj[1:])
    if vwgt is None:
        vwgt = np.ones(n, dtype=np.int32)
    return Graph(xadj, dst.astype(np.int32), np.asarray(vwgt, dtype=np.int32), ww, name)


def grid2d(nx: int, ny: int) -> Graph:
    """nx-by-ny 5-point grid; vertex (i, j) has id i*ny + j; unit weights."""
    ids = np.arange(nx * ny, dtype=np.int64).reshape(nx, ny)
    us, vs = [], []
    us.append(ids[:, :-1].ravel()); vs.append(ids[:, 1:].ravel())
    us.append(ids[:-1, :].ravel()); vs.append(ids[1:, :].ravel())
    return csr_from_edges(nx * ny, np.concatenate(us), np.concatenate(vs),
                          name=f"grid2d_{nx}x{ny}")


def stencil27(nx: int, ny: int, nz: int) -> Graph:
    """3-D 27-point stencil mesh; vertex (x, y, z) has id (x*ny + y)*nz + z.

    Every vertex is joined to all of its up to 26 neighbours; unit weights.
    Built row by row in sorted order, so no global sort is needed.
    """
    n = nx * ny * nz
    xs = np.arange(nx)
    ys = np.arange(ny)
    zs = np.arange(nz)
    X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
    X = X.ravel(); Y = Y.ravel(); Z = Z.ravel()
    deg = np.zeros(n, dtype=np.int64)
    offs = [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)
            if (dx, dy, dz) != (0, 0, 0)]
    # offsets in increasing neighbour-id order: id delta = (dx*ny + dy)*nz + dz
    offs.sort(key=lambda o: (o[0] * ny + o[1]) * nz + o[2])
    valid = []
    for dx, dy, dz in offs:
        ok = ((X + dx >= 0) & (X + dx < nx) & (Y + dy >= 0) & (Y + dy < ny)
              & (Z + dz >= 0) & (Z + dz < nz))
        valid.append(ok)
        deg += ok
    xadj = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=xadj[1:])
    adj = np.empty(int(xadj[-1]), dtype=np.int32)
    pos = xadj[:-1].copy()
    vid = np.arange(n, dtype=np.int64)
    for (dx, dy, dz), ok in zip(offs, valid):
        delta = (dx * ny + dy) * nz + dz
        idx = np.nonzero(ok)[0]
        adj[pos[idx]] = (vid[idx] + delta).astype(np.int32)
        pos[idx] += 1
    nnz = int(xadj[-1])
    return Graph(xadj, adj, np.ones(n, dtype=np.int32), np.ones(nnz, dtype=np.int32),
                 name=f"stencil27_{nx}x{ny}x{nz}")


def rmat(scale: int, edge_factor: int, seed: int, a=0.57, b=0.19, c=0.19,
         wmax: int = 16, permute: bool = True) -> Graph:
    """R-MAT graph, symmetrised, deduplicated, self-loop free, isolated kept.

    Each of ``edge_factor * 2**scale`` samples picks one quadrant per bit
    level. A level draw is a 16-bit uniform; one 64-bit SplitMix64 output
    yields four levels. Quadrant thresholds are a, a+b, a+b+c quantised to
    1/65536. Edge i of the sorted unique canonical list gets weight
    1 + floor(stream(seed_w, i) * wmax / 2**64). Ids are relabelled by a
    seeded permutation (argsort of random keys), so hubs are not at low ids.
    """
    n = 1 << scale
    ns = edge_factor * n
    s_bits = subseed(seed, 2)
    ta = int(round(a * 65536)); tb = int(round((a + b) * 65536)); tc = int(round((a + b + c) * 65536))
    import torch  # multithreaded elementwise bit work; same integers as numpy
    src = torch.zeros(ns, dtype=torch.int64)
    dst = torch.zeros(ns, dtype=torch.int64)
    sample = np.arange(ns, dtype=np.uint64)
    nwords = (scale + 3) // 4
    for wi in range(nwords):
        with np.errstate(over="ignore"):
            x = torch.from_numpy(stream(s_bits, sample * np.uint64(nwords) + np.uint64(wi)).view(np.int64))
        for j in range(4):
            lvl = wi * 4 + j
            if lvl >= scale:
                break
            r = (x >> (16 * j)) & 0xFFFF  # the 16-bit field; masking undoes the sign of the shift
            bit_src = (r >= tb).to(torch.int64)            # quadrants c, d -> lower half
            bit_dst = (((r >= ta) & (r < tb)) | (r >= tc)).to(torch.int64)  # b, d -> right
            src |= bit_src << lvl
            dst |= bit_dst << lvl
        del x
    del sample
    src = src.numpy(); dst = dst.numpy()
    keep = src != dst
    src = src[keep]; dst = dst[keep]
    lo = np.minimum(src, dst); hi = np.maximum(src, dst)
    del src, dst
    key = np.unique(lo * np.int64(n) + hi)
    lo = key // n; hi = key % n
    del key
    m = lo.shape[0]
    w = (1 + uniform_below(stream(subseed(seed, 3), np.arange(m, dtype=np.uint64)), wmax)).astype(np.int32)
    if permute:
        keys = stream(subseed(seed, 4), np.arange(n, dtype=np.uint64))
        perm = np.argsort(keys, kind="stable").astype(np.int64)  # new id of old vertex i = position
        newid = np.empty(n, dtype=np.int64)
        newid[perm] = np.arange(n, dtype=np.int64)
        lo = newid[lo]; hi = newid[hi]
        a2 = np.minimum(lo, hi); b2 = np.maximum(lo, hi)
        lo, hi = a2, b2
    return csr_from_edges(n, lo, hi, w, name=f"rmat_s{scale}_ef{edge_factor}")


def rgg_radius(n: int, mean_degree: float = 10.0) -> float:
    """Radius r with (n-1)*(pi r^2 - 8 r^3/3 + r^4/2) = mean_degree (bisection).

    The bracket is the exact probability that two uniform points of the unit
    square lie within distance r (r <= 1).
    """
    target = mean_degree / max(n - 1, 1)
    lo, hi = 0.0, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        p = math.pi * mid * mid - 8.0 * mid ** 3 / 3.0 + mid ** 4 / 2.0
        if p < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def rgg(n: int, seed: int, mean_degree: float = 10.0) -> Graph:
    """2-D random geometric graph in the unit square.

    Points are 53-bit uniforms from two SplitMix64 streams. Edges join pairs
    at distance <= r. Vertices are ordered by (cell row, cell column,
    generation index) over a grid of cells of side >= r.
    """
    r = rgg_radius(n, mean_degree)
    idx = np.arange(n, dtype=np.uint64)
    xs = (stream(subseed(seed, 5), idx) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
    ys = (stream(subseed(seed, 6), idx) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
    ncell = max(1, int(1.0 / r))
    cx = np.minimum((xs * ncell).astype(np.int64), ncell - 1)
    cy = np.minimum((ys * ncell).astype(np.int64), ncell - 1)
    order = np.lexsort((np.arange(n), cx, cy))
    xs = xs[order]; ys = ys[order]; cx = cx[order]; cy = cy[order]
    cell = cy * ncell + cx
    cstart = np.searchsorted(cell, np.arange(ncell * ncell + 1))
    us, vs = [], []
    r2 = r * r
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            ny_ = cy + dy; nx_ = cx + dx
            ok = (ny_ >= 0) & (ny_ < ncell) & (nx_ >= 0) & (nx_ < ncell)
            vid = np.nonzero(ok)[0]
            nc = ny_[vid] * ncell + nx_[vid]
            s = cstart[nc]; e = cstart[nc + 1]
            cnt = e - s
            rep = np.repeat(vid, cnt)
            base = np.repeat(s - np.cumsum(np.concatenate([[0], cnt[:-1]])), cnt)
            cand = base + np.arange(rep.shape[0])
            keep = cand > rep
            rep = rep[keep]; cand = cand[keep]
            d2 = (xs[rep] - xs[cand]) ** 2 + (ys[rep] - ys[cand]) ** 2
            keep = d2 <= r2
            us.append(rep[keep]); vs.append(cand[keep])
    u = np.concatenate(us); v = np.concatenate(vs)
    return csr_from_edges(n, u, v, name=f"rgg_{n}")


def random_partition(n: int, k: int, seed: int) -> np.ndarray:
    """P0[v] = floor(stream(seed, v) * k / 2**64): seeded uniform part per vertex."""
    return uniform_below(stream(seed, np.arange(n, dtype=np.uint64)), k).astype(np.int32)


def validate_csr(g: Graph) -> None:
    """Raise ValueError unless g is a symmetric, simple, positively weighted CSR graph."""
    n = g.n
    xadj = g.xadj
    if xadj[0] != 0 or np.any(np.diff(xadj) < 0):
        raise ValueError("xadj not monotone from 0")
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(xadj))
    dst = g.adjncy.astype(np.int64)
    if dst.size and (dst.min() < 0 or dst.max() >= n):
        raise ValueError("adjncy out of range")
    if np.any(src == dst):
        raise ValueError("self-loop")
    if np.any(g.vwgt < 1) or np.any(g.adjwgt < 1):
        raise ValueError("non-positive weight")
    key = src * n + dst
    rkey = dst * n + src
    o1 = np.argsort(key)
    if np.any(np.diff(key[o1]) == 0):
        raise ValueError("parallel edge")
    o2 = np.argsort(rkey)
    if not np.array_equal(key[o1], rkey[o2]):
        raise ValueError("not symmetric")
    if not np.array_equal(g.adjwgt[o1], g.adjwgt[o2]):
        raise ValueError("asymmetric weights")


def small_random_graph(n: int, p_edge: float, seed: int, wmax: int = 1, vwmax: int = 1) -> Graph:
    """Erdos-Renyi-like tiny graph for exhaustive tests (SplitMix64 driven)."""
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    if not pairs:
        return csr_from_edges(n, np.zeros(0, np.int64), np.zeros(0, np.int64),
                              vwgt=np.ones(n, np.int32))
    x = stream(seed, np.arange(len(pairs), dtype=np.uint64))
    thr = np.uint64(min(int(p_edge * 2.0 ** 64), (1 << 64) - 1))
    sel = x < thr
    u = np.array([p[0] for p, s in zip(pairs, sel) if s], dtype=np.int64)
    v = np.array([p[1] for p, s in zip(pairs, sel) if s], dtype=np.int64)
    w = (1 + uniform_below(stream(subseed(seed, 3), np.arange(u.shape[0], dtype=np.uint64)), wmax)
         ).astype(np.int32) if u.shape[0] else np.zeros(0, np.int32)
    vw = (1 + uniform_below(stream(subseed(seed, 4), np.arange(n, dtype=np.uint64)), vwmax)).astype(np.int32)
    return csr_from_edges(n, u, v, w, vwgt=vw, name=f"er_{n}_{seed}")


# ------------------------------------------------------------- workloads --
# Recipes of the batched and serving workloads (sizes, k and seeds only).

def rgg_batch_spec(count: int = 512, nmin: int = 1000, nmax: int = 200000, seed: int = 77):
    """(n, k, seed) per graph: n log-uniform on [nmin, nmax], k uniform in
    {2, 4, ..., 128}. Graph i is ``rgg(n, seed)`` with P_0 =
    ``random_partition(n, k, seed)``."""
    u = stream(seed, np.arange(2 * count, dtype=np.uint64))
    frac = (u[:count] >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    ns = np.exp(np.log(nmin) + (np.log(nmax) - np.log(nmin)) * frac).astype(np.int64)
    ks = np.array([2, 4, 8, 16, 32, 64, 128])[uniform_below(u[count:], 7)]
    return [(int(ns[i]), int(ks[i]), seed * 100003 + i) for i in range(count)]


# Graph pool of the serving workload: 2-D grids (unit weights) and R-MAT
# graphs (scale, edge factor, seed; weights 1..16).
SERVE_POOL = [("grid", 64), ("grid", 128), ("grid", 256), ("grid", 512), ("grid", 1024),
              ("rmat", 12, 8, 41), ("rmat", 14, 16, 42), ("rmat", 16, 8, 43), ("rmat", 18, 16, 44),
              ("rmat", 20, 16, 45)]


def serve_pool_graph(spec) -> Graph:
    if spec[0] == "grid":
        return grid2d(spec[1], spec[1])
    return rmat(spec[1], spec[2], spec[3])


def serve_job_specs(count: int, seed: int = 99):
    """Per-job draws of the serving mix: half 2-D grids with side uniform in
    [64, 1024] (unit weights), half R-MAT graphs with scale uniform in
    [12, 20], edge factor uniform in [8, 16] and a graph seed of their own
    (weights 1..16); k uniform in [2, 256]; a partition seed per job.
    Returns (graph spec, k, seed) per job; ``serve_pool_graph(spec)`` draws
    the graph."""
    u = stream(subseed(seed, 10), np.arange(5 * count, dtype=np.uint64))
    kind = uniform_below(u[:count], 2)
    side = 64 + uniform_below(u[count:2 * count], 1024 - 64 + 1)
    scale = 12 + uniform_below(u[2 * count:3 * count], 9)
    ef = 8 + uniform_below(u[3 * count:4 * count], 9)
    ks = 2 + uniform_below(u[4 * count:], 255)
    out = []
    for i in range(count):
        spec = ("grid", int(side[i])) if kind[i] == 0 else ("rmat", int(scale[i]), int(ef[i]), 5000 + i)
        out.append((spec, int(ks[i]), 1000 + i))
    return out


def serve_jobs(count: int, seed: int = 99):
    """(pool index, k uniform in [2, 256], seed) per job."""
    u = stream(seed, np.arange(2 * count, dtype=np.uint64))
    gi = uniform_below(u[:count], len(SERVE_POOL))
    ks = 2 + uniform_below(u[count:], 255)
    return [(int(gi[i]), int(ks[i]), 1000 + i) for i in range(count)]


def arrivals(rate: float, count: int, seed: int) -> np.ndarray:
    """Poisson process: exponential gaps of mean 1/rate, first arrival at 0."""
    u = (stream(seed, np.arange(count, dtype=np.uint64)) >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    gaps = -np.log1p(-u) / rate
    return np.cumsum(gaps) - gaps[0]
