// Jet refinement on gfx950: Jetlp with the afterburner (Algorithm 4), weak and
// strong rebalancing (Algorithm 5 and the strong variant of Section 4.2.2),
// synchronous move application, and the refinement loop of Algorithm 3 run by
// device-side controllers -- for one graph or for a batch of graphs.
//
// Design (one MI355X):
//  * A batch is one block-diagonal union graph: graph g owns the vertices
//    [voff_g, voff_g + n_g), the global parts [poff_g, poff_g + k_g) and the
//    tiles [t0_g, t0_g + ntiles_g). No edge joins two graphs, so every
//    connectivity, gain and loss is the graph's own, and each graph keeps its
//    own controller, counters and iteration kind. One launch sequence per
//    iteration serves every graph; a single graph is a batch of one.
//  * Connectivity conn(v, .) is rebuilt per pass in LDS. Vertices are binned
//    by degree: <= 32 -> 4- or 8-lane groups, <= 1024 -> one wave, larger ->
//    one block. Each group owns a dense int32 table of k + 1 entries;
//    neighbours add their edge weight with LDS atomics, then read-and-clear
//    the entry of their own part with an atomic exchange, so every adjacent
//    part is seen exactly once and the table is left zero. Integer sums are
//    exact in any order; argmax ties break by part id, so no result depends
//    on scheduling.
//  * Per-vertex Jetlp state is one 8-byte record (P_s, P_d + in-X flag, F), so
//    the afterburner's neighbour gather is a single load.
//  * Rebalancing orders evictions by (loss slot, vertex id): a per-(part,
//    slot) weight histogram fixes each oversized part's cut-off slot; inside
//    it, per-(part, tile) weight sums locate the one tile where the residual
//    is reached, and an ordered scan of that tile fixes the last evicted id.
//  * A controller block per graph ends each iteration (best tracking, trace,
//    the next kind) and counts the graphs of each kind; the other kernels
//    exit at once when no graph needs them, so iterations are enqueued in
//    chunks with one host sync per chunk.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "jet_device.h"
#include "jet_internal.h"

namespace jet {

// ------------------------------------------------------------- graph views --

__device__ __forceinline__ int graph_of(const KArgs &a, int v) { return a.vg ? a.vg[v] : 0; }

// Kernels on the hot path are built twice: B = false for one graph (graph 0
// everywhere, its fields loaded once per lane at kernel start), B = true for
// a batch (graph looked up per vertex).
template <bool B>
__device__ __forceinline__ int gof(const KArgs &a, int v)
{
    return B ? a.vg[v] : 0;
}

// Count row of the current iteration: [improved-and-going-on, Jetlp, Jetrw, Jetrs].
__device__ __forceinline__ const int32_t *count_row(const KArgs &a) { return a.cnt + CNT_ROW + (a.it & 1) * 4; }
__device__ __forceinline__ bool any_kind(const KArgs &a, int kind) { return count_row(a)[kind] > 0; }
__device__ __forceinline__ bool any_rb(const KArgs &a)
{
    const int32_t *r = count_row(a);
    return r[KIND_RW] + r[KIND_RS] > 0;
}
__device__ __forceinline__ bool any_active(const KArgs &a)
{
    const int32_t *r = count_row(a);
    return r[KIND_LP] + r[KIND_RW] + r[KIND_RS] > 0;
}
__device__ __forceinline__ bool is_rb(int kind) { return kind == KIND_RW || kind == KIND_RS; }

// Per-lane copy of the fields of a vertex's graph that a kernel reads. A lane
// reloads it only when it reaches a vertex of another graph: lanes walk
// contiguous stretches of a batch, and a single graph loads it once. Fields a
// kernel does not use are never loaded.
struct GV {
    int g = -1;
    int kind = 0, lp_id = 0, cn = 0, cd = 1, k = 0, poff = 0, voff = 0, nB = 0, copy = 0;
    int64_t W = 0;
    uint64_t hs = 0;  // Jetrw hash seed of the iteration: mix64(seed ^ (level * 2^32 + t))
    __device__ __forceinline__ void at(const KArgs &a, int gg)
    {
        if (gg == g) return;
        g = gg;
        const Ctl *c = a.ctl + gg;
        kind = c->kind;
        lp_id = c->lp_id;
        cn = c->c_num;
        cd = c->c_den;
        k = c->k;
        poff = c->poff;
        voff = c->voff;
        nB = c->nB;
        copy = c->copy_best;
        W = c->W;
        hs = mix64(c->seed ^ (((uint64_t)(uint32_t)c->level << 32) + (uint64_t)(uint32_t)c->t));
    }
    template <bool B>
    __device__ __forceinline__ void sel(const KArgs &a, int gg)
    {
        if (B) at(a, gg);
    }
};

// Counters are summed modulo 2^64 (signed values and the digest alike).
__device__ __forceinline__ void stat_add(const KArgs &a, int g, int row, uint64_t val)
{
    if (val)
        atomicAdd((unsigned long long *)&a.bstat[((int64_t)g * NSTAT + row) * NSHARD + (blockIdx.x & (NSHARD - 1))],
                  (unsigned long long)val);
}

// Up to three iteration counters of the graph a lane is visiting; reaching
// another graph adds the previous graph's counts to its shards.
template <int R0, int R1 = -1, int R2 = -1>
struct GAcc {
    static constexpr int r1 = R1, r2 = R2;
    int g = -1;
    uint64_t c0 = 0, c1 = 0, c2 = 0;
    __device__ __forceinline__ void flush(const KArgs &a)
    {
        if (g >= 0) {
            stat_add(a, g, R0, c0);
            if (R1 >= 0) stat_add(a, g, R1, c1);
            if (R2 >= 0) stat_add(a, g, R2, c2);
        }
        c0 = 0;
        c1 = 0;
        c2 = 0;
    }
    __device__ __forceinline__ void to(const KArgs &a, int gg)
    {
        if (gg != g) {
            flush(a);
            g = gg;
        }
    }
    template <bool B>
    __device__ __forceinline__ void sel(const KArgs &a, int gg)
    {
        if (B) to(a, gg);
    }
};

// End of a kernel (whole block): when every counting lane is in the same
// graph (always for one graph) the counts are summed over the block and added
// once per row; otherwise every lane adds its own.
template <class Acc>
__device__ void acc_finish(const KArgs &a, Acc &acc)
{
    __shared__ int s_lo, s_hi;
    __shared__ uint64_t s_red[BLOCK / 64];
    if (threadIdx.x == 0) {
        s_lo = INT_MAX;
        s_hi = -1;
    }
    __syncthreads();
    if (acc.g >= 0) {
        atomicMin(&s_lo, acc.g);
        atomicMax(&s_hi, acc.g);
    }
    __syncthreads();
    const int lo = s_lo, hi = s_hi;
    __syncthreads();
    if (hi < 0) return;
    if (lo == hi) {
        const uint64_t t0 = block_sum<BLOCK>(acc.c0, s_red);
        uint64_t t1 = 0, t2 = 0;
        if (Acc::r1 >= 0) t1 = block_sum<BLOCK>(acc.c1, s_red);
        if (Acc::r2 >= 0) t2 = block_sum<BLOCK>(acc.c2, s_red);
        acc.c0 = t0;
        acc.c1 = t1;
        acc.c2 = t2;
        acc.g = threadIdx.x == 0 ? lo : -1;
    }
    acc.flush(a);
}

// List entries a worker visits, in steps of `unit` (64 for the wave-batched
// role, else 1): one graph interleaves the workers; a batch gives each worker
// one contiguous stretch, so its vertices fall in few graphs.
struct Walk {
    int first, end, step;
    int32_t *wq = nullptr;  // batch work queue counter (NULL: static walk)
    int tile = 0;           // entries per tile
};

// Work-queue slots of the batch row kernels (one queue per kernel and
// class, two banks selected by the iteration's launch parity; the controller
// clears the next iteration's bank). (Per-XCD sub-queues over contiguous
// eighths of a list, with stealing, measured slower than one counter.)
enum WqSlot {
    WQ_GAIN = 0,     // + small class (1, 2)
    WQ_GAIN2 = 3,    // + class of the wave role (1..4)
    WQ_LOSS = 8,     // + small class
    WQ_LOSS2 = 11,   // + class of the wave role
    WQ_AFTER_S = 16, WQ_AFTER_M = 17, WQ_DCUT_S = 18, WQ_DCUT_M = 19,
    NQ = 20
};
constexpr int NQC = NQ;  // counters per bank
static_assert(NQC <= BLOCK, "the controller's block clears a bank in one pass");

// Blocks are dispatched to the 8 XCDs round robin (block b on XCD b mod 8).
// Renumbered so that the blocks of one XCD form a contiguous range, its
// waves walk neighbouring stretches of a list and its L2 holds their
// neighbours' parts. Identity unless the grid is a multiple of 8.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    if (nb % NXCD) return b;
    return (b % NXCD) * (nb / NXCD) + b / NXCD;
}
template <bool B>
__device__ __forceinline__ Walk walk(int cnt, int worker, int nworkers, int unit)
{
    Walk w;
    if (!B) {
        w.first = worker * unit;
        w.end = cnt;
        w.step = nworkers * unit;
    } else {
        int64_t chunk = ((int64_t)cnt + nworkers - 1) / nworkers;
        chunk = (chunk + unit - 1) / unit * unit;
        int64_t lo = (int64_t)worker * chunk;
        lo = lo < cnt ? lo : cnt;
        const int64_t hi = lo + chunk < cnt ? lo + chunk : cnt;
        w.first = (int)lo;
        w.end = (int)hi;
        w.step = unit;
    }
    return w;
}

// Walk of a batch row kernel: with a work queue, waves take tiles of
// wtile * unit list entries from the slot's counter until the list is
// exhausted (load balance across graphs and degree mixes); otherwise the
// static walk.
template <bool B>
__device__ __forceinline__ Walk walk_q(const KArgs &a, int cnt, int worker, int nworkers, int unit, int slot)
{
    if (B && a.wq && a.wtile > 0) {
        Walk w;
        w.first = 0;
        w.end = cnt;
        w.step = unit;
        w.wq = a.wq + (a.it & 1) * NQC + slot;
        w.tile = a.wtile * unit;
        return w;
    }
    return walk<B>(cnt, worker, nworkers, unit);
}

// Contiguous range [lo, hi) of `cnt` items for block `b` of `nb`.
__device__ __forceinline__ void block_chunk(int cnt, int b, int nb, int &lo, int &hi)
{
    int64_t chunk = ((int64_t)cnt + nb - 1) / nb;
    chunk = (chunk + BLOCK - 1) / BLOCK * BLOCK;
    int64_t l = (int64_t)b * chunk;
    l = l < cnt ? l : cnt;
    lo = (int)l;
    hi = (int)(l + chunk < cnt ? l + chunk : cnt);
}

// Range of the per-vertex passes: one graph walks its vertex ids; a batch
// walks its class lists, which hold only the vertices of graphs still
// running once they have been compacted.
template <bool B>
__device__ __forceinline__ void flat_range(const KArgs &a, int &lo, int &hi)
{
    block_chunk(B ? a.binoff[NCLS] : a.n, blockIdx.x, gridDim.x, lo, hi);
}
template <bool B>
__device__ __forceinline__ int flat_vertex(const KArgs &a, int i)
{
    return B ? a.bins[i] : i;
}

// CSR entry loads. NT: where each wave-wide load covers whole cache lines of
// the row (a wave or a block walking one row), the entries are streamed with
// non-temporal loads so that the stream does not evict the gathered part
// array from L2 (on a power-law graph with random ids this cuts the pass's
// L2 misses by a third). Lane groups that take a row a few entries per
// instruction re-read each line from L1 and keep ordinary loads.
template <bool NT = false>
__device__ __forceinline__ int ld_adj(const KArgs &a, int64_t i)
{
    return NT ? __builtin_nontemporal_load(a.adj + i) : a.adj[i];
}
template <bool NT = false>
__device__ __forceinline__ int ld_ew(const KArgs &a, int64_t i)
{
    return a.ew ? (NT ? __builtin_nontemporal_load(a.ew + i) : a.ew[i]) : 1;
}

// Part of neighbour u for a gather: the byte copy when it exists.
__device__ __forceinline__ int gpart(const KArgs &a, int u) { return a.P8 ? (int)a.P8[u] : (int)a.P[u]; }

// Packed (old, new) part of a vertex: set when a move is selected (new =
// destination) and when P_iter changes (old = new = P_iter).
__device__ __forceinline__ void mq_set(const KArgs &a, int v, int oldp, int newp)
{
    if (a.P8) ((uint16_t *)a.mq)[v] = (uint16_t)((oldp << 8) | newp);
    else ((uint32_t *)a.mq)[v] = ((uint32_t)oldp << 16) | (uint32_t)newp;
}
__device__ __forceinline__ uint32_t mq_load(const KArgs &a, int u)
{
    return a.P8 ? (uint32_t)((const uint16_t *)a.mq)[u] : ((const uint32_t *)a.mq)[u];
}

// Compact Jetlp record of a vertex for the afterburner's gathers, when
// every part id fits a byte (k <= 256): P_s in bits 31..24, P_d (in X) or
// P_s (not in X; P_d != P_s in X) in bits 23..16, F saturated to int16 in
// bits 15..0. A saturated F still orders exactly against any F that is not
// beyond the same bound; the full F is read only in that rare case.
__device__ __forceinline__ void rq_set(const KArgs &a, int v, int ps, int pq, int F)
{
    const int fs = F > 32767 ? 32767 : (F < -32768 ? -32768 : F);
    ((uint32_t *)a.rq)[v] = ((uint32_t)ps << 24) | ((uint32_t)pq << 16) | ((uint32_t)fs & 0xFFFFu);
}

// Jetlp record of vertex v in rec's layout (x = P_s << 16 | (in X ? P_d + 1 :
// 0), y = F for a vertex of X), from rq and Fx when those replace rec.
__device__ __forceinline__ int2 own_rec(const KArgs &a, int v)
{
    if (!a.rq) return a.rec[v];
    const uint32_t q = a.rq[v];
    const int ps = (int)(q >> 24), pq = (int)((q >> 16) & 0xFFu);
    if (pq == ps) return make_int2(ps << 16, 0);
    return make_int2((ps << 16) | (pq + 1), a.Fx[v]);
}

__device__ __forceinline__ int degree_class(int64_t d)
{
    return d == 0 ? CLS_Z : (d <= S_MAXDEG ? CLS_S : (d <= S2_MAXDEG ? CLS_S2 : (d <= M_MAXDEG ? CLS_M : CLS_L)));
}

// ------------------------------------------------------------------ set-up --

// Copies P_0, clears per-vertex state, sums vertex weights and part weights,
// counts degree classes per block (for the ordered bins) and checks part ids,
// vertex weights and row offsets. Vertex weights and the digest go to
// counter rows 0 and 1 of the graph. Blocks own contiguous ranges.
__global__ __launch_bounds__(BLOCK) void k_init_vertices(KArgs a, const int32_t *part_in, int32_t *blkcnt)
{
    extern __shared__ int32_t s_w[];  // [k] block-partial part weights (one graph)
    __shared__ int32_t s_cls[NCLS];
    const bool single = a.vg == nullptr;
    if (single)
        for (int p = threadIdx.x; p < a.k; p += BLOCK) s_w[p] = 0;
    if (threadIdx.x < NCLS) s_cls[threadIdx.x] = 0;
    __syncthreads();
    int lo, hi;
    block_chunk(a.n, blockIdx.x, gridDim.x, lo, hi);
    GV gv;
    GAcc<0, 1> acc;
    int bad = 0;
    for (int v = lo + threadIdx.x; v < hi; v += BLOCK) {
        const int g = graph_of(a, v);
        gv.at(a, g);
        acc.to(a, g);
        int p = part_in[v];
        if (p < 0 || p >= gv.k) {
            a.ctl[g].bad_part = 1;
            p = 0;
        } else if (a.best != part_in) {
            a.best[v] = p;
        }
        a.P[v] = (uint16_t)p;
        if (a.P8) a.P8[v] = (uint8_t)p;
        mq_set(a, v, p, p);
        a.dest[v] = -1;
        a.lock[v] = -1;
        a.slot[v] = 255;
        const int vwv = a.vw ? a.vw[v] : 1;
        if (vwv < 1) bad = 1;
        int64_t d = a.xadj[v + 1] - a.xadj[v];
        if (d < 0) {
            bad = 1;
            d = 0;
        }
        atomicAdd(&s_cls[degree_class(d)], 1);
        if (single) atomicAdd(&s_w[p], vwv);
        else atomicAdd((unsigned long long *)&a.w[gv.poff + p], (unsigned long long)(int64_t)vwv);
        acc.c0 += vwv;
        acc.c1 += mix64(((uint64_t)(uint32_t)(v - gv.voff) << 32) | (uint32_t)p);
    }
    if (bad) a.cnt[1] = 1;
    acc_finish(a, acc);
    __syncthreads();
    if (threadIdx.x < NCLS) blkcnt[blockIdx.x * NCLS + threadIdx.x] = s_cls[threadIdx.x];
    if (single)
        for (int p = threadIdx.x; p < a.k; p += BLOCK)
            if (s_w[p]) atomicAdd((unsigned long long *)&a.w[p], (unsigned long long)(int64_t)s_w[p]);
}

// Row marks (see row_marks) for the edge passes.
__global__ __launch_bounds__(BLOCK) void k_row_marks(const int64_t *xadj, int n, int64_t nmark, int32_t *mark)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < nmark; i += (int64_t)gridDim.x * BLOCK) {
        const int64_t e = i * MARK;
        int lo = 0, hi = n + 1;  // largest lo with xadj[lo] <= e (xadj[0] = 0 <= e)
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (xadj[mid] <= e) lo = mid;
            else hi = mid;
        }
        mark[i] = lo;
    }
}

// Edge pass: cut of P_0 and total edge weight (counter rows 2 and 3),
// neighbour-range / self-loop / weight checks. Block b takes the entries of
// row-mark interval b, [b * MARK, (b + 1) * MARK). When the interval's rows
// fit in LDS, their offsets, parts (and graphs) are staged there and the
// entries are read coalesced, four per thread in flight, each finding its row
// by a binary search in LDS. Otherwise each thread takes runs of 16
// consecutive entries: it finds the run's first row between the interval's
// rows, loads the 16 entries and gathers their parts at once, then walks the
// rows.
constexpr int EDGE_ROWS = 1024;
__global__ __launch_bounds__(BLOCK) void k_init_edges(KArgs a, int64_t nnz, const int32_t *mark, int64_t nmark)
{
    __shared__ int64_t s_x[EDGE_ROWS + 1];
    __shared__ int32_t s_p[EDGE_ROWS];
    __shared__ int32_t s_g[EDGE_ROWS];
    const int n = a.n;
    if (n < 1) return;  // callers refine no empty graph
    GAcc<2, 3> acc;
    int bad = 0;
    for (int64_t blk = blockIdx.x; blk * MARK < nnz; blk += gridDim.x) {
        const int64_t e_lo = blk * MARK, e_hi = e_lo + MARK < nnz ? e_lo + MARK : nnz;
        // rows r_lo..r_hi hold the interval on well-formed offsets; both stay
        // in [0, n) on malformed ones (the checks below and the vertex pass
        // flag those)
        int r_lo = mark[blk];
        int r_hi = blk + 1 < nmark ? mark[blk + 1] : n - 1;
        if (r_hi > n - 1) r_hi = n - 1;
        if (r_lo > r_hi) r_lo = r_hi;
        const int nr = r_hi - r_lo + 1;
        if (nr <= EDGE_ROWS) {
            for (int i = threadIdx.x; i <= nr; i += BLOCK) {
                s_x[i] = a.xadj[r_lo + i];
                if (i < nr) {
                    s_p[i] = a.P[r_lo + i];
                    s_g[i] = graph_of(a, r_lo + i);
                }
            }
            __syncthreads();
            constexpr int U = 4;
            for (int64_t e0 = e_lo + threadIdx.x; e0 < e_hi; e0 += (int64_t)BLOCK * U) {
                int u[U], wt[U], pu[U];
#pragma unroll
                for (int j = 0; j < U; j++) {
                    const int64_t e = e0 + (int64_t)j * BLOCK;
                    u[j] = e < e_hi ? ld_adj(a, e) : -1;
                    wt[j] = e < e_hi ? ld_ew(a, e) : 1;
                }
#pragma unroll
                for (int j = 0; j < U; j++) pu[j] = (u[j] >= 0 && u[j] < n) ? gpart(a, u[j]) : -1;
#pragma unroll
                for (int j = 0; j < U; j++) {
                    const int64_t e = e0 + (int64_t)j * BLOCK;
                    if (e >= e_hi) continue;
                    int lo = 0, hi = nr;  // largest lo with s_x[lo] <= e
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (s_x[mid] <= e) lo = mid;
                        else hi = mid;
                    }
                    const int v = r_lo + lo;
                    if (u[j] < 0 || u[j] >= n || u[j] == v || wt[j] < 1) {
                        bad = 1;
                        continue;
                    }
                    acc.to(a, s_g[lo]);
                    acc.c1 += wt[j];
                    if (u[j] > v && pu[j] != s_p[lo]) acc.c0 += wt[j];
                }
            }
            __syncthreads();
            continue;
        }
        constexpr int RUN = 16;
        for (int64_t e0 = e_lo + (int64_t)threadIdx.x * RUN; e0 < e_hi; e0 += (int64_t)BLOCK * RUN) {
            const int64_t e1 = e0 + RUN < e_hi ? e0 + RUN : e_hi;
            int lo = r_lo, hi = r_hi + 1;  // largest lo with xadj[lo] <= e0
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (a.xadj[mid] <= e0) lo = mid;
                else hi = mid;
            }
            int u[RUN], wt[RUN], pu[RUN];
#pragma unroll
            for (int j = 0; j < RUN; j++) {
                const int64_t e = e0 + j;
                u[j] = e < e1 ? ld_adj(a, e) : -1;
                wt[j] = e < e1 ? ld_ew(a, e) : 1;
            }
#pragma unroll
            for (int j = 0; j < RUN; j++) pu[j] = (u[j] >= 0 && u[j] < n) ? gpart(a, u[j]) : -1;
            int v = lo;
            int64_t vend = a.xadj[v + 1];
            int pv = a.P[v];
            acc.to(a, graph_of(a, v));
#pragma unroll
            for (int j = 0; j < RUN; j++) {
                const int64_t e = e0 + j;
                if (e >= e1) break;
                while (e >= vend && v < n - 1) {
                    v++;
                    vend = a.xadj[v + 1];
                    pv = a.P[v];
                    acc.to(a, graph_of(a, v));
                }
                if (u[j] < 0 || u[j] >= n || u[j] == v || wt[j] < 1) {
                    bad = 1;
                    continue;
                }
                acc.c1 += wt[j];
                if (u[j] > v && pu[j] != pv) acc.c0 += wt[j];
            }
        }
    }
    if (bad) a.cnt[1] = 1;
    acc_finish(a, acc);
}

// Largest weighted degree (one wave per vertex, int64 sums): run only when a
// graph's total edge weight reaches 2^31, to check that every vertex's
// weighted degree, which bounds its connectivities, gains and losses, stays
// below 2^31.
__global__ __launch_bounds__(BLOCK) void k_wdeg_max(const int64_t *xadj, const int32_t *ew, int n,
                                                    unsigned long long *out)
{
    const int lane = threadIdx.x & 63;
    const int nw = gridDim.x * (BLOCK / 64);
    int64_t best = 0;
    for (int v = blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6); v < n; v += nw) {
        const int64_t s = xadj[v], e = xadj[v + 1];
        int64_t sum = 0;
        for (int64_t i = s + lane; i < e; i += 64) sum += ew[i];
        sum = gsum<64>(sum);
        best = sum > best ? sum : best;
    }
    if (lane == 0 && best > 0) atomicMax(out, (unsigned long long)best);
}

// Per graph (one wave each): totals of the set-up counters into the controller.
__global__ __launch_bounds__(64) void k_init_reduce(KArgs a)
{
    const int g = blockIdx.x;
    const int64_t *b = a.bstat + (int64_t)g * NSTAT * NSHARD + threadIdx.x;
    const int64_t ws = gsum<64>(b[0 * NSHARD]);
    const uint64_t dg = gsum<64>((uint64_t)b[1 * NSHARD]);
    const int64_t cut = gsum<64>(b[2 * NSHARD]);
    const int64_t ews = gsum<64>(b[3 * NSHARD]);
    if (threadIdx.x == 0) {
        Ctl *c = a.ctl + g;
        c->wsum = ws;
        c->digest = dg;
        c->cut = cut;
        c->ewsum = ews;
    }
}

// Block offsets per degree class: exclusive scan over blocks, class-major, so
// every class lists its vertices in ascending id. Totals land after the
// nblk * NCLS offsets.
__global__ __launch_bounds__(BLOCK) void k_bin_scan(int32_t *blkcnt, int nblk)
{
    __shared__ int32_t s_scan[BLOCK / 64];
    int32_t base = 0;
    for (int c = 0; c < NCLS; c++) {
        int32_t carry = 0;
        for (int b0 = 0; b0 < nblk; b0 += BLOCK) {
            const int b = b0 + threadIdx.x;
            const int32_t x = b < nblk ? blkcnt[b * NCLS + c] : 0;
            int32_t tot;
            const int32_t ex = block_excl_scan<BLOCK>(x, s_scan, tot);
            if (b < nblk) blkcnt[b * NCLS + c] = base + carry + ex;
            carry += tot;
        }
        if (threadIdx.x == 0) blkcnt[nblk * NCLS + c] = carry;
        base += carry;
    }
}

// Ordered fill of the class lists; same grid and ranges as k_init_vertices.
__global__ __launch_bounds__(BLOCK) void k_fill_bins(KArgs a, const int32_t *blkoff, int32_t *bins)
{
    __shared__ int32_t s_scan[BLOCK / 64];
    int lo, hi;
    block_chunk(a.n, blockIdx.x, gridDim.x, lo, hi);
    int32_t run[NCLS];
#pragma unroll
    for (int c = 0; c < NCLS; c++) run[c] = blkoff[blockIdx.x * NCLS + c];
    for (int base = lo; base < hi; base += BLOCK) {
        const int v = base + threadIdx.x;
        int cls = -1;
        if (v < hi) cls = degree_class(a.xadj[v + 1] - a.xadj[v]);
#pragma unroll
        for (int c = 0; c < NCLS; c++) {
            int32_t tot;
            const int32_t pos = block_excl_scan<BLOCK>((int32_t)(cls == c), s_scan, tot);
            if (cls == c) bins[run[c] + pos] = v;
            run[c] += tot;
        }
    }
}

// Batch compaction: class counts and ordered class lists of the vertices of
// graphs still running (same grid and ranges in both kernels).
__global__ __launch_bounds__(BLOCK) void k_bin_count_active(KArgs a, int32_t *blkcnt)
{
    __shared__ int32_t s_cls[NCLS];
    if (threadIdx.x < NCLS) s_cls[threadIdx.x] = 0;
    __syncthreads();
    GV gv;
    int lo, hi;
    block_chunk(a.n, blockIdx.x, gridDim.x, lo, hi);
    for (int v = lo + threadIdx.x; v < hi; v += BLOCK) {
        gv.at(a, graph_of(a, v));
        if (gv.kind == KIND_DONE) continue;
        atomicAdd(&s_cls[degree_class(a.xadj[v + 1] - a.xadj[v])], 1);
    }
    __syncthreads();
    if (threadIdx.x < NCLS) blkcnt[blockIdx.x * NCLS + threadIdx.x] = s_cls[threadIdx.x];
}

__global__ __launch_bounds__(BLOCK) void k_fill_bins_active(KArgs a, const int32_t *blkoff, int32_t *bins)
{
    __shared__ int32_t s_scan[BLOCK / 64];
    GV gv;
    int lo, hi;
    block_chunk(a.n, blockIdx.x, gridDim.x, lo, hi);
    int32_t run[NCLS];
#pragma unroll
    for (int c = 0; c < NCLS; c++) run[c] = blkoff[blockIdx.x * NCLS + c];
    for (int base = lo; base < hi; base += BLOCK) {
        const int v = base + threadIdx.x;
        int cls = -1;
        if (v < hi) {
            gv.at(a, graph_of(a, v));
            if (gv.kind != KIND_DONE) cls = degree_class(a.xadj[v + 1] - a.xadj[v]);
        }
#pragma unroll
        for (int c = 0; c < NCLS; c++) {
            int32_t tot;
            const int32_t pos = block_excl_scan<BLOCK>((int32_t)(cls == c), s_scan, tot);
            if (cls == c) bins[run[c] + pos] = v;
            run[c] += tot;
        }
    }
}

// -------------------------------------------------------------- controller --

// Oversized parts A = {w > o}, valid destinations B = {w <= sigma} listed in
// ascending id, and a cleared (part, slot) histogram, for graph g. Whole
// block calls.
// wreg: when not null, the caller's registers hold w(p) for p = threadIdx.x +
// j * BLOCK, j < WREG (k <= WREG * BLOCK).
constexpr int WREG = 4;

__device__ void rb_prepare(const KArgs &a, int g, const int64_t *wreg = nullptr)
{
    __shared__ int32_t s_scan[BLOCK / 64];
    Ctl *c = a.ctl + g;
    const int64_t o = c->o, sigma = c->sigma;
    const int k = c->k, poff = c->poff;
    int32_t carry = 0, nA = 0;
    for (int base = 0; base < k; base += BLOCK) {
        const int p = base + threadIdx.x;
        int inA = 0, inB = 0;
        if (p < k) {
            const int64_t wp = wreg ? wreg[base / BLOCK] : a.w[poff + p];
            inA = wp > o;
            inB = wp <= sigma;
            a.isA[poff + p] = (uint8_t)inA;
            a.isB[poff + p] = (uint8_t)inB;
        }
        int32_t tot;
        const int32_t pos = block_excl_scan<BLOCK>((int32_t)inB, s_scan, tot);
        if (inB) a.Blist[poff + carry + pos] = p;
        carry += tot;
        int32_t ta;
        block_excl_scan<BLOCK>((int32_t)inA, s_scan, ta);
        nA += ta;
    }
    for (int i = threadIdx.x; i < k * NSLOT; i += BLOCK) a.hist[(int64_t)poff * NSLOT + i] = 0;
    if (threadIdx.x == 0) {
        c->nB = carry;
        c->nA = nA;
    }
}

__device__ __forceinline__ void clear_accumulators(Ctl *c)
{
    c->nX = 0;
    c->nM = 0;
    c->dcut = 0;
    c->moved_w = 0;
    c->ddigest = 0;
}

// Decides the kind of the next iteration from the loop state (thread 0):
// stop after stall_limit iterations without a new best (or at max_iters);
// Jetlp while balanced, else Jetrw for b_max iterations, then Jetrs. The
// stall counter rises here, at the start of every iteration.
__device__ __forceinline__ int ctl_next(Ctl &cc)
{
    int kind;
    if (cc.done || cc.stall >= cc.stall_limit || (cc.max_iters > 0 && cc.t >= cc.max_iters)) {
        cc.done = 1;
        kind = KIND_DONE;
    } else {
        cc.stall++;
        if (cc.balanced) {
            kind = KIND_LP;
            // without locks (ablation) Jetlp ids advance by 2, so no stamp
            // ever equals the previous id and nothing is locked
            cc.lp_id += (cc.flags & JET_F_LP_NO_LOCKS) ? 2 : 1;
            cc.wcount = 0;
            cc.n_lp++;
        } else if (cc.wcount < cc.bmax) {
            kind = KIND_RW;
            cc.wcount++;
            cc.n_rw++;
        } else {
            kind = KIND_RS;
            cc.wcount++;
            cc.n_rs++;
        }
    }
    cc.kind = kind;
    clear_accumulators(&cc);
    return kind;
}

// Whole-block part of starting graph g's next iteration: clear its counter
// shards and, for rebalancing, build A, B and clear its histogram.
__device__ __forceinline__ void begin_iteration(const KArgs &a, int g, int kind, const int64_t *wreg = nullptr)
{
    for (int i = threadIdx.x; i < NSTAT * NSHARD; i += BLOCK) a.bstat[(int64_t)g * NSTAT * NSHARD + i] = 0;
    if (is_rb(kind)) rb_prepare(a, g, wreg);
}

// Adds graph g's next kind (and whether its best must be copied) to the
// count row of launch `it`.
__device__ __forceinline__ void count_next(const KArgs &a, int it, int next, int copy)
{
    if (next == KIND_DONE) {
        atomicAdd(&a.cnt[CNT_DONE], 1);
        return;
    }
    int32_t *row = a.cnt + CNT_ROW + (it & 1) * 4;
    atomicAdd(&row[next], 1);
    if (copy) atomicAdd(&row[0], 1);
}

// Per graph (one block each): loop state after the set-up passes (W, o and
// sigma are already set), then the first iteration's kind.
__global__ __launch_bounds__(BLOCK) void k_ctl_setup(KArgs a)
{
    __shared__ uint64_t s_red[BLOCK / 64];
    __shared__ int s_next;
    const int g = blockIdx.x;
    Ctl *c = a.ctl + g;
    const int k = c->k, poff = c->poff;
    uint64_t m = 0;
    for (int p = threadIdx.x; p < k; p += BLOCK) {
        const uint64_t x = (uint64_t)a.w[poff + p];
        m = x > m ? x : m;
        a.wbest[poff + p] = a.w[poff + p];
    }
    m = block_max_u64<BLOCK>(m, s_red);
    if (threadIdx.x == 0) {
        Ctl cc = *c;
        cc.maxw = (int64_t)m;
        cc.balanced = (int64_t)m <= cc.o;
        cc.bal_best = cc.balanced;
        cc.cut_best = cc.cut;
        cc.maxw_best = cc.maxw;
        const int next = ctl_next(cc);  // iteration 0
        *c = cc;
        s_next = next;
        count_next(a, a.it, next, 0);
    }
    __syncthreads();
    begin_iteration(a, g, s_next);
}

// Per graph (one block each): end of an iteration. Sums the counter shards,
// applies Algorithm 3's best / stall rules, writes the trace record, decides
// the next iteration and starts it.
__global__ __launch_bounds__(BLOCK) void k_ctl_end(KArgs a)
{
    __shared__ uint64_t s_red[BLOCK / 64];
    __shared__ int s_improved, s_next;
    // this launch's count row has been read by every kernel of the iteration:
    // clear it for the iteration after next
    if (blockIdx.x == 0 && threadIdx.x < 4) a.cnt[CNT_ROW + (a.it & 1) * 4 + threadIdx.x] = 0;
    // the connectivity rows listed for rebuilding were rebuilt by now
    if (blockIdx.x == 0 && threadIdx.x == 4) a.cnt[CNT_TFAIL] = 0;
    // the next iteration's work-queue counters (its bank was last used two
    // iterations ago)
    if (a.wq && blockIdx.x == 0 && threadIdx.x < NQC) a.wq[((a.it + 1) & 1) * NQC + threadIdx.x] = 0;
    const int g = blockIdx.x;
    Ctl *c = a.ctl + g;
    // thread 0 fetches the whole state while the block reads the part
    // weights and counter shards: one round trip before the decision
    Ctl cc;
    if (threadIdx.x == 0) cc = *c;
    const int kind = c->kind;
    if (kind == KIND_DONE) return;
    const int k = c->k, poff = c->poff;
    // the NSHARD shards of each counter row: one lane of the first wave each
    int64_t sx = 0, sm = 0, sdc = 0, smw = 0, se = 0, sr = 0, sv = 0;
    if (threadIdx.x < NSHARD) {
        const int64_t *b = a.bstat + (int64_t)g * NSTAT * NSHARD + threadIdx.x;
        sx = b[ST_X * NSHARD];
        sm = b[ST_M * NSHARD];
        sdc = b[ST_DCUT * NSHARD];
        smw = b[ST_MW * NSHARD];
        se = b[ST_DIG * NSHARD];
        if (kind == KIND_LP) {
            sr = b[ST_R * NSHARD];
            sv = b[ST_V * NSHARD];
        }
    }
    int64_t pe = 0;
    if (threadIdx.x < NSHARD && kind == KIND_LP) pe = a.bstat[(int64_t)g * NSTAT * NSHARD + ST_E * NSHARD + threadIdx.x];
    // part weights stay in registers for the best copy and the rebalancing set-up
    const bool inreg = k <= WREG * BLOCK;
    int64_t wreg[WREG];
#pragma unroll
    for (int j = 0; j < WREG; j++) {
        const int p = threadIdx.x + j * BLOCK;
        wreg[j] = (inreg && p < k) ? a.w[poff + p] : 0;
    }
    uint64_t m = 0;
    if (inreg) {
#pragma unroll
        for (int j = 0; j < WREG; j++) m = (uint64_t)wreg[j] > m ? (uint64_t)wreg[j] : m;
    } else {
        for (int p = threadIdx.x; p < k; p += BLOCK) {
            const uint64_t x = (uint64_t)a.w[poff + p];
            m = x > m ? x : m;
        }
    }
    m = block_max_u64<BLOCK>(m, s_red);
    int64_t px = 0, pm = 0, pdc = 0, pmw = 0, pr = 0, pv = 0;
    uint64_t pdg = 0;
    if (threadIdx.x < NSHARD) {
        px = gsum<NSHARD>(sx);
        pm = gsum<NSHARD>(sm);
        pdc = gsum<NSHARD>(sdc);
        pmw = gsum<NSHARD>(smw);
        pdg = gsum<NSHARD>((uint64_t)se);
        if (kind == KIND_LP) {
            pe = gsum<NSHARD>(pe);
            pr = gsum<NSHARD>(sr);
            pv = gsum<NSHARD>(sv);
        }
    }
    if (threadIdx.x == 0) {
        const int64_t maxw = (int64_t)m;
        cc.nX = (int)px;
        cc.nM = (int)pm;
        cc.dcut = pdc;
        cc.moved_w = pmw;
        cc.ddigest = pdg;
        cc.prof_e += pe;
        cc.prof_r += pr;
        cc.prof_v += pv;
        cc.cut += cc.dcut;
        cc.digest += cc.ddigest;
        cc.maxw = maxw;
        const int bal = maxw <= cc.o;
        cc.balanced = bal;
        int improved = 0;
        if (bal) {
            if (!cc.bal_best) {
                // a balanced partition always replaces an imbalanced best
                improved = 1;
                cc.bal_best = 1;
                cc.cut_best = cc.cut;
                cc.maxw_best = maxw;
                cc.stall = 0;
            } else if (cc.cut < cc.cut_best) {
                // only a gain beyond the tolerance phi restarts the count
                if ((int64_t)cc.phi_den * cc.cut < (int64_t)cc.phi_num * cc.cut_best) cc.stall = 0;
                improved = 1;
                cc.cut_best = cc.cut;
                cc.maxw_best = maxw;
            }
        } else if (!cc.bal_best && maxw < cc.maxw_best) {
            improved = 1;
            cc.maxw_best = maxw;
            cc.cut_best = cc.cut;
            cc.stall = 0;
        }
        cc.copy_best = improved;
        if (g == 0 && a.kinds && cc.t < KIND_LOG) a.kinds[cc.t] = (int8_t)kind;
        if (a.trace && cc.t < cc.trace_cap) {
            jet_trace_rec r;
            r.level = cc.level;
            r.t = cc.t;
            r.kind = kind;
            r.nX = cc.nX;
            r.nM = cc.nM;
            r.stall = cc.stall;
            r.wcount = cc.wcount;
            r.balanced = bal;
            r.moved_w = cc.moved_w;
            r.cut = cc.cut;
            r.maxw = maxw;
            r.best_cut = cc.cut_best;
            r.digest = cc.digest;
            a.trace[(int64_t)cc.trace_off + cc.t] = r;
        }
        cc.t++;
        const int next = ctl_next(cc);
        *c = cc;
        s_improved = improved;
        s_next = next;
        count_next(a, a.it + 1, next, improved);
    }
    __syncthreads();
    if (s_improved) {
        if (inreg) {
#pragma unroll
            for (int j = 0; j < WREG; j++) {
                const int p = threadIdx.x + j * BLOCK;
                if (p < k) a.wbest[poff + p] = wreg[j];
            }
        } else {
            for (int p = threadIdx.x; p < k; p += BLOCK) a.wbest[poff + p] = a.w[poff + p];
        }
    }
    begin_iteration(a, g, s_next, inreg ? wreg : nullptr);
}

// After the loop: P_iter into P_best for graphs whose last iteration improved
// the best (earlier improvements were copied by the next cut-delta pass).
__global__ __launch_bounds__(BLOCK) void k_copy_best(KArgs a)
{
    if (!a.vg && !a.ctl->copy_best) return;
    GV gv;
    int lo, hi;
    block_chunk(a.n, blockIdx.x, gridDim.x, lo, hi);
    for (int v = lo + threadIdx.x; v < hi; v += BLOCK) {
        gv.at(a, graph_of(a, v));
        if (gv.copy) a.best[v] = a.P[v];
    }
}

// P_iter widened into a caller's int32 array (JET_F_RETURN_ITER).
__global__ __launch_bounds__(BLOCK) void k_copy_iter(KArgs a, int32_t *out)
{
    for (int v = blockIdx.x * BLOCK + threadIdx.x; v < a.n; v += gridDim.x * BLOCK) out[v] = a.P[v];
}

// Single-step entry points (one graph): force one iteration of `kind` at
// index t. For Jetlp, lock flags become stamps of the previous Jetlp (id 0).
__global__ __launch_bounds__(BLOCK) void k_force_step(KArgs a, int kind, int t, const uint8_t *locked)
{
    Ctl *c = a.ctl;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c->kind = kind;
        c->t = t;
        c->lp_id = 1;
        clear_accumulators(c);
        for (int i = 0; i < 8; i++) a.cnt[CNT_ROW + i] = 0;
        a.cnt[CNT_ROW + (a.it & 1) * 4 + kind] = 1;
    }
    if (locked)
        for (int v = blockIdx.x * BLOCK + threadIdx.x; v < a.n; v += gridDim.x * BLOCK) a.lock[v] = locked[v] ? 0 : -1;
    if (blockIdx.x == 0) {
        __syncthreads();
        begin_iteration(a, 0, kind);
    }
}

// Defaults of the step outputs for vertices no row kernel visits (isolated).
__global__ __launch_bounds__(BLOCK) void k_step_defaults(KArgs a, const int32_t *part)
{
    for (int v = blockIdx.x * BLOCK + threadIdx.x; v < a.n; v += gridDim.x * BLOCK) {
        if (a.dbg_F) {
            a.dbg_F[v] = INT64_MIN;
            a.dbg_cs[v] = 0;
            a.dbg_F2[v] = 0;
            a.dbg_pd[v] = part[v];
        }
        if (a.dbg_loss) {
            a.dbg_loss[v] = INT64_MIN;
            a.dbg_slot[v] = -1;
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_lp_outputs(KArgs a, uint8_t *inX, uint8_t *move)
{
    for (int v = blockIdx.x * BLOCK + threadIdx.x; v < a.n; v += gridDim.x * BLOCK) {
        const bool iso = a.xadj[v + 1] == a.xadj[v];
        inX[v] = iso ? 0 : (uint8_t)((own_rec(a, v).x & 0xFFFF) != 0);
        move[v] = a.dest[v] >= 0;
    }
}

// ------------------------------------------------------ connectivity core --

// Group of G lanes gathers the neighbours of a row (deg <= G*R) into table
// `tab` and reads every adjacent part's total back exactly once: on return
// pu[r] is the part of neighbour slot r (-1 if none) and cu[r] its
// connectivity for the first lane that claimed it, else 0. The table is left
// all-zero.
template <int G, int R>
__device__ __forceinline__ void group_conn_row(const KArgs &a, int64_t s, int deg, int gl, int32_t *tab, int (&pu)[R],
                                               int (&cu)[R])
{
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int idx = gl + r * G;
        pu[r] = -1;
        if (idx < deg) {
            const int u = ld_adj<G == 64>(a, s + idx);
            const int wt = ld_ew<G == 64>(a, s + idx);
            pu[r] = gpart(a, u);
            atomicAdd(&tab[pu[r]], wt);
        }
    }
    lds_fence_wave();
#pragma unroll
    for (int r = 0; r < R; r++) cu[r] = pu[r] >= 0 ? atomicExch(&tab[pu[r]], 0) : 0;
    lds_fence_wave();
}

// The two halves of group_conn_row for rows of unit edge weights, so that a
// group can have two rows' loads in flight: conn_load gathers a row's
// neighbour parts (slot r of lane gl is entry gl + r * G; -1 beyond the row),
// conn_claim adds them into `tab` and reads every adjacent part's total back
// exactly once (cu as in group_conn_row).
template <int G, int R>
__device__ __forceinline__ void conn_load(const KArgs &a, int64_t s, int deg, int gl, int (&pu)[R])
{
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int idx = gl + r * G;
        pu[r] = idx < deg ? ld_adj(a, s + idx) : -1;
    }
#pragma unroll
    for (int r = 0; r < R; r++) pu[r] = pu[r] >= 0 ? gpart(a, pu[r]) : -1;
}

template <int R>
__device__ __forceinline__ void conn_claim(int32_t *tab, const int (&pu)[R], int (&cu)[R])
{
#pragma unroll
    for (int r = 0; r < R; r++)
        if (pu[r] >= 0) atomicAdd(&tab[pu[r]], 1);
    lds_fence_wave();
#pragma unroll
    for (int r = 0; r < R; r++) cu[r] = pu[r] >= 0 ? atomicExch(&tab[pu[r]], 0) : 0;
    lds_fence_wave();
}

// Group of G lanes adds the neighbours of a row (deg <= G*R) into `tab`; all
// R neighbour ids (and weights) of a lane are loaded before its dependent
// part gathers. The caller reads the table back.
template <int G, int R>
__device__ __forceinline__ void group_fill_row(const KArgs &a, int64_t s, int deg, int gl, int32_t *tab)
{
    int u[R], w[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int idx = gl + r * G;
        u[r] = idx < deg ? ld_adj<G == 64>(a, s + idx) : -1;
        w[r] = idx < deg ? ld_ew<G == 64>(a, s + idx) : 0;
    }
#pragma unroll
    for (int r = 0; r < R; r++) u[r] = u[r] >= 0 ? gpart(a, u[r]) : -1;
#pragma unroll
    for (int r = 0; r < R; r++)
        if (u[r] >= 0) atomicAdd(&tab[u[r]], w[r]);
    lds_fence_wave();
}

// Parts a whole-wave row reads back by scanning its k-entry table (and
// clearing what it finds) rather than claiming entry by entry: the scan is
// k / 64 LDS reads per lane against one atomic exchange per row entry.
constexpr int WAVE_SCAN_KMAX = 1024;

// Wave-batched driver of the small-row role. Lanes first inspect 64 list
// entries at once (coalesced loads of the id, row offsets and per-vertex
// state); the entries that need row work are queued in LDS and handed to the
// wave's groups of G lanes. Metadata round trips are paid once per 64
// vertices instead of once per vertex, and skipped vertices cost no group
// time.
struct Meta {
    int v, ps, deg, aux, g;
    int64_t s;
};

// Next tile [lo, hi) of a queued walk: lane 0 takes it, the wave shares it
// (lo >= hi once the list is exhausted).
__device__ __forceinline__ void walk_grab(const Walk &w, int &lo, int &hi)
{
    int b = 0;
    if ((threadIdx.x & 63) == 0) b = atomicAdd(w.wq, w.tile);
    b = __shfl(b, 0, 64);
    lo = b < w.end ? b : w.end;
    hi = b + w.tile < w.end ? b + w.tile : w.end;
}

template <int G, class Pre, class Row>
__device__ __forceinline__ void wave_batched(const int32_t *list, Walk w, int32_t *q, Pre pre, Row row,
                                             int unit = 64)
{
    const int lane = threadIdx.x & 63, grp = lane / G, gl = lane & (G - 1);
    int lo = w.first, hi = w.end;
    if (w.wq) walk_grab(w, lo, hi);
    for (;;) {
    if (lo >= hi) break;
    for (int base = lo; base < hi; base += w.step) {
        const int i = base + lane;
        Meta m{0, 0, 0, 0, 0, 0};
        bool act = false;
        if (lane < unit && i < hi) {
            m.v = list ? list[i] : i;  // no list: entry i is vertex i
            act = pre(m);
        }
        const uint64_t mask = __ballot(act);
        if (act) q[__popcll(mask & ((1ull << lane) - 1ull))] = lane;
        lds_fence_wave();
        const int nact = __popcll(mask);
        for (int sb = 0; sb < nact; sb += 64 / G) {
            const int slot = sb + grp;
            const bool has = slot < nact;
            const int src = q[has ? slot : 0];
            Meta t;
            t.v = __shfl(m.v, src, 64);
            t.ps = __shfl(m.ps, src, 64);
            t.deg = __shfl(m.deg, src, 64);
            t.aux = __shfl(m.aux, src, 64);
            t.g = __shfl(m.g, src, 64);
            t.s = __shfl(m.s, src, 64);
            if (has) row(t, gl);
        }
        lds_fence_wave();
    }
    if (!w.wq) break;
    walk_grab(w, lo, hi);
    if (lo >= hi) break;
    }
}

// wave_batched with two queued rows per group and round: the row callback
// gets both, each with a flag saying whether it exists, and can issue the
// loads of both before the LDS work of either. Every lane takes part in the
// shuffles (a shuffle under a divergent mask could read an inactive lane).
template <int G, class Pre, class Row2>
__device__ __forceinline__ void wave_batched2(const int32_t *list, Walk w, int32_t *q, Pre pre, Row2 row2)
{
    constexpr int NG = 64 / G;
    const int lane = threadIdx.x & 63, grp = lane / G, gl = lane & (G - 1);
    for (int base = w.first; base < w.end; base += w.step) {
        const int i = base + lane;
        Meta m{0, 0, 0, 0, 0, 0};
        bool act = false;
        if (i < w.end) {
            m.v = list ? list[i] : i;
            act = pre(m);
        }
        const uint64_t mask = __ballot(act);
        if (act) q[__popcll(mask & ((1ull << lane) - 1ull))] = lane;
        lds_fence_wave();
        const int nact = __popcll(mask);
        for (int sb = 0; sb < nact; sb += 2 * NG) {
            const int s0 = sb + grp, s1 = sb + NG + grp;
            const bool h0 = s0 < nact, h1 = s1 < nact;
            const int c0 = q[h0 ? s0 : 0], c1 = q[h1 ? s1 : 0];
            Meta t0, t1;
            t0.v = __shfl(m.v, c0, 64);
            t0.ps = __shfl(m.ps, c0, 64);
            t0.deg = __shfl(m.deg, c0, 64);
            t0.aux = __shfl(m.aux, c0, 64);
            t0.g = __shfl(m.g, c0, 64);
            t0.s = __shfl(m.s, c0, 64);
            t1.v = __shfl(m.v, c1, 64);
            t1.ps = __shfl(m.ps, c1, 64);
            t1.deg = __shfl(m.deg, c1, 64);
            t1.aux = __shfl(m.aux, c1, 64);
            t1.g = __shfl(m.g, c1, 64);
            t1.s = __shfl(m.s, c1, 64);
            if (!h0) t0.deg = 0;
            if (!h1) t1.deg = 0;
            row2(t0, h0, t1, h1, gl);
        }
        lds_fence_wave();
    }
}

// List entries a wave inspects per visit when every queued row takes the
// whole wave (wave_batched<64>): 64, halved while the list would leave waves
// idle, so short lists still spread over the grid.
__device__ __forceinline__ int wave_unit(int cnt, int nwaves)
{
    int u = 64;
    while (u > 1 && (int64_t)u * nwaves > cnt) u >>= 1;
    return u;
}

// Rows longer than a group walk their entries in rounds of U per lane: all
// U neighbour ids (and weights) are loaded, then all U dependent gathers are
// issued, so a lane has U loads in flight instead of one.
constexpr int UROW = 8;

// Whole block gathers the neighbours of v into `tab`.
__device__ __forceinline__ void block_fill(const KArgs &a, int v, int32_t *tab)
{
    const int64_t s = a.xadj[v], e = a.xadj[v + 1];
    for (int64_t base = s + threadIdx.x; base < e; base += (int64_t)BLOCK * UROW) {
        int u[UROW], w[UROW], p[UROW];
#pragma unroll
        for (int j = 0; j < UROW; j++) {
            const int64_t i = base + (int64_t)j * BLOCK;
            u[j] = i < e ? ld_adj<true>(a, i) : -1;
            w[j] = i < e ? ld_ew<true>(a, i) : 0;
        }
#pragma unroll
        for (int j = 0; j < UROW; j++) p[j] = u[j] >= 0 ? gpart(a, u[j]) : -1;
#pragma unroll
        for (int j = 0; j < UROW; j++)
            if (p[j] >= 0) atomicAdd(&tab[p[j]], w[j]);
    }
    __syncthreads();
}

// Largest-connectivity key: connectivity in the high word, ~part in the low
// word, so ties go to the smaller part id.
__device__ __forceinline__ uint64_t conn_key(int c, int p) { return ((uint64_t)(uint32_t)c << 32) | (uint32_t)(~p); }

// Rows of at most TINY entries are taken one per lane, by the lane that
// inspects them in the wave-batched drivers: the row's neighbour parts sit in
// registers and are compared pairwise, so no lane group, LDS table or
// reduction is spent on a row of a few entries (most rows of a power-law
// graph).
constexpr int TINY = 8;

// Connectivity of such a row (deg <= T): calls f(p, conn(v, p)) once for
// every adjacent part p != ps and returns conn(v, ps).
template <int T, class F>
__device__ __forceinline__ int tiny_conn(const KArgs &a, int64_t s, int deg, int ps, F f)
{
    int p[T], w[T];
#pragma unroll
    for (int j = 0; j < T; j++) {
        p[j] = j < deg ? ld_adj(a, s + j) : -1;
        w[j] = j < deg ? ld_ew(a, s + j) : 0;
    }
#pragma unroll
    for (int j = 0; j < T; j++) p[j] = p[j] >= 0 ? gpart(a, p[j]) : -1;
    int cs = 0;
#pragma unroll
    for (int j = 0; j < T; j++) cs += p[j] == ps ? w[j] : 0;
#pragma unroll
    for (int j = 0; j < T; j++) {
        if (p[j] < 0 || p[j] == ps) continue;
        bool first = true;
        int c = w[j];
#pragma unroll
        for (int i = 0; i < T; i++) {
            if (i < j) first = first && p[i] != p[j];
            else if (i > j) c += p[i] == p[j] ? w[i] : 0;
        }
        if (first) f(p[j], c);  // the first slot of a part reports its whole sum
    }
    return cs;
}

// -------------------------------------------------------------- Jetlp gain --

// Writes rec[v]; returns whether v passes the first filter (a destination
// exists and F >= 0 or -F < floor(c * conn(v, P_s))).
__device__ __forceinline__ bool gain_finish(const KArgs &a, int v, int ps, uint64_t best, int cs, int cn, int cd)
{
    int2 r;
    r.x = ps << 16;
    r.y = 0;
    bool inx = false;
    int pd = ps;
    int64_t F = INT64_MIN;
    if (best) {
        pd = (int)(~(uint32_t)best);
        const int f = (int)(best >> 32) - cs;
        const int64_t thr = ((int64_t)cn * cs) / cd;
        inx = f >= 0 || -(int64_t)f < thr;
        r.y = f;
        F = f;
        if (inx) r.x |= pd + 1;
    }
    if (a.rq) {
        rq_set(a, v, ps, inx ? pd : ps, r.y);
        if (inx) a.Fx[v] = r.y;
    } else {
        a.rec[v] = r;
    }
    if (a.dbg_F) {
        a.dbg_F[v] = F;
        a.dbg_cs[v] = cs;
        a.dbg_pd[v] = pd;
    }
    return inx;
}

__device__ __forceinline__ void gain_locked(const KArgs &a, int v, int ps)
{
    if (a.rq) rq_set(a, v, ps, ps, 0);
    else a.rec[v] = make_int2(ps << 16, 0);
    if (a.dbg_F) {
        a.dbg_F[v] = INT64_MIN;
        a.dbg_cs[v] = 0;
        a.dbg_pd[v] = ps;
    }
}

typedef GAcc<ST_V, ST_R, ST_E> GainPre;  // visited vertices, unlocked rows, their CSR entries
typedef GAcc<ST_X> CountX;

template <bool B, int G, int R>
__device__ void gain_groups(const KArgs &a, int cls, int32_t *tab, int gid, int ngroups, GV &gv, GainPre &pacc,
                            CountX &racc)
{
    const int gl = threadIdx.x & (G - 1);
    const int32_t *list = a.bins + a.binoff[cls];
    const Walk w = walk<B>(a.binoff[cls + 1] - a.binoff[cls], gid, ngroups, 1);
    for (int i = w.first; i < w.end; i += w.step) {
        const int v = list[i];
        const int g = gof<B>(a, v);
        gv.sel<B>(a, g);
        if (gv.kind != KIND_LP) continue;
        const int ps = a.P[v];
        if (gl == 0) {
            pacc.sel<B>(a, g);
            pacc.c0++;
        }
        if (a.lock[v] == gv.lp_id - 1) {
            if (gl == 0) gain_locked(a, v, ps);
            continue;
        }
        const int64_t s = a.xadj[v];
        const int deg = (int)(a.xadj[v + 1] - s);
        if (gl == 0) {
            pacc.c1++;
            pacc.c2 += deg;
        }
        int pu[R], cu[R];
        group_conn_row<G, R>(a, s, deg, gl, tab, pu, cu);
        uint64_t best = 0;
        int cs = 0;
#pragma unroll
        for (int r = 0; r < R; r++) {
            if (cu[r] > 0) {
                if (pu[r] == ps) cs += cu[r];
                else {
                    const uint64_t k2 = conn_key(cu[r], pu[r]);
                    best = k2 > best ? k2 : best;
                }
            }
        }
        best = gmax_u64<G>(best);
        cs = gsum<G>(cs);
        if (gl == 0) {
            racc.sel<B>(a, g);
            racc.c0 += gain_finish(a, v, ps, best, cs, gv.cn, gv.cd);
        }
    }
}

template <bool B>
__device__ void gain_blocks(const KArgs &a, int cls, int32_t *tab, int bid, int nblocks, GV &gv, GainPre &pacc,
                            CountX &racc)
{
    __shared__ uint64_t s_red[BLOCK / 64];
    __shared__ int32_t s_red32[BLOCK / 64];
    const int32_t *list = a.bins + a.binoff[cls];
    const Walk w = walk<B>(a.binoff[cls + 1] - a.binoff[cls], bid, nblocks, 1);
    for (int i = w.first; i < w.end; i += w.step) {
        const int v = list[i];
        const int g = gof<B>(a, v);
        gv.sel<B>(a, g);
        if (gv.kind != KIND_LP) continue;
        const int ps = a.P[v];
        if (threadIdx.x == 0) {
            pacc.sel<B>(a, g);
            pacc.c0++;
        }
        if (a.lock[v] == gv.lp_id - 1) {
            if (threadIdx.x == 0) gain_locked(a, v, ps);
            continue;
        }
        if (threadIdx.x == 0) {
            pacc.c1++;
            pacc.c2 += a.xadj[v + 1] - a.xadj[v];
        }
        block_fill(a, v, tab);
        uint64_t best = 0;
        int cs = 0;
        for (int p = threadIdx.x; p < gv.k; p += BLOCK) {
            const int c = tab[p];
            if (c) {
                tab[p] = 0;
                if (p == ps) cs = c;
                else {
                    const uint64_t k2 = conn_key(c, p);
                    best = k2 > best ? k2 : best;
                }
            }
        }
        best = block_max_u64<BLOCK>(best, s_red);
        cs = block_sum<BLOCK>(cs, s_red32);
        if (threadIdx.x == 0) {
            racc.sel<B>(a, g);
            racc.c0 += gain_finish(a, v, ps, best, cs, gv.cn, gv.cd);
        }
    }
}

// Role layout of the LDS-table kernels: one kernel per role (small-row
// groups, waves, blocks), so each keeps its own register budget; a.tmap says
// which classes a role serves. Group tables are padded to k + 1 ints so the
// tables of neighbouring groups start in different LDS banks.
template <bool B, int ROLE, int GS, int RS, int CL, bool PAIR = false>
__device__ __forceinline__ void gain_body(const KArgs &a, int nblk)
{
    extern __shared__ int32_t lds[];
    const int stride = a.k + 1;
    GV pv, rv;
    GainPre pacc;
    CountX racc;
    if (!B) {
        pv.at(a, 0);
        rv.at(a, 0);
        pacc.to(a, 0);
        racc.to(a, 0);
    }
    if (ROLE == 1) {
        // groups of G lanes (rows of up to G * R entries) over one small
        // class, wave-batched. CL = NCLS: blocks [0, gS) take class S with
        // (GS, RS), the next gS2 blocks class S2 with groups of 8 lanes.
        const int ng = BLOCK / GS;
        for (int i = threadIdx.x; i < ng * stride; i += BLOCK) lds[i] = 0;
        __syncthreads();
        int32_t *q = lds + ng * stride + (threadIdx.x >> 6) * 64;
        auto body = [&](auto g_c, auto r_c, int cl, int bid, int nb) {
            constexpr int G = decltype(g_c)::value, R = decltype(r_c)::value;
            if (a.tmap[cl] != ROLE) return;
            int32_t *tab = lds + (threadIdx.x / G) * stride;
            if (!B && CL != NCLS) bid = xcd_block(bid, nb);
            const int wid = bid * (BLOCK / 64) + (threadIdx.x >> 6), nwaves = nb * (BLOCK / 64);
            const int32_t *list = (!B && cl == CLS_S && a.sident) ? nullptr : a.bins + a.binoff[cl];
            const Walk wk = walk_q<B>(a, a.binoff[cl + 1] - a.binoff[cl], wid, nwaves, 64, WQ_GAIN + cl);
            auto pre = [&](Meta &m) -> bool {
                    m.g = gof<B>(a, m.v);
                    pv.sel<B>(a, m.g);
                    if (pv.kind != KIND_LP) return false;
                    // part, lock stamp and row bounds in one round trip
                    m.ps = a.P[m.v];
                    const int lk = a.lock[m.v];
                    const int64_t x0 = a.xadj[m.v], x1 = a.xadj[m.v + 1];
                    pacc.sel<B>(a, m.g);
                    pacc.c0++;
                    if (lk == pv.lp_id - 1) {
                        gain_locked(a, m.v, m.ps);
                        return false;
                    }
                    m.s = x0;
                    m.deg = (int)(x1 - x0);
                    pacc.c1++;
                    pacc.c2 += m.deg;
                    if (!PAIR && m.deg <= TINY) {
                        uint64_t best = 0;
                        const int cs = tiny_conn<TINY>(a, m.s, m.deg, m.ps, [&](int p, int c) {
                            const uint64_t k2 = conn_key(c, p);
                            best = k2 > best ? k2 : best;
                        });
                        racc.sel<B>(a, m.g);
                        racc.c0 += gain_finish(a, m.v, m.ps, best, cs, pv.cn, pv.cd);
                        return false;
                    }
                    return true;
                };
            auto row = [&](const Meta &t, int gl) {
                    int pu[R], cu[R];
                    group_conn_row<G, R>(a, t.s, t.deg, gl, tab, pu, cu);
                    uint64_t best = 0;
                    int cs = 0;
#pragma unroll
                    for (int r = 0; r < R; r++) {
                        if (cu[r] > 0) {
                            if (pu[r] == t.ps) cs += cu[r];
                            else {
                                const uint64_t k2 = conn_key(cu[r], pu[r]);
                                best = k2 > best ? k2 : best;
                            }
                        }
                    }
                    best = gmax_u64<G>(best);
                    cs = gsum<G>(cs);
                    if (gl == 0) {
                        rv.sel<B>(a, t.g);
                        racc.sel<B>(a, t.g);
                        racc.c0 += gain_finish(a, t.v, t.ps, best, cs, rv.cn, rv.cd);
                    }
                };
            if (PAIR && cl == CLS_S && !a.ew) {
                // two rows per group and round, both rows' parts in flight at once
                auto row2 = [&](const Meta &t0, bool h0, const Meta &t1, bool h1, int gl) {
                    int p0[R], p1[R], cu[R];
                    conn_load<G, R>(a, t0.s, t0.deg, gl, p0);
                    conn_load<G, R>(a, t1.s, t1.deg, gl, p1);
                    auto finish = [&](const Meta &t, const int (&pu)[R]) {
                        conn_claim<R>(tab, pu, cu);
                        uint64_t best = 0;
                        int cs = 0;
#pragma unroll
                        for (int r = 0; r < R; r++) {
                            if (cu[r] > 0) {
                                if (pu[r] == t.ps) cs += cu[r];
                                else {
                                    const uint64_t k2 = conn_key(cu[r], pu[r]);
                                    best = k2 > best ? k2 : best;
                                }
                            }
                        }
                        best = gmax_u64<G>(best);
                        cs = gsum<G>(cs);
                        if (gl == 0) {
                            rv.sel<B>(a, t.g);
                            racc.sel<B>(a, t.g);
                            racc.c0 += gain_finish(a, t.v, t.ps, best, cs, rv.cn, rv.cd);
                        }
                    };
                    if (h0) finish(t0, p0);
                    if (h1) finish(t1, p1);
                };
                wave_batched2<G>(list, wk, q, pre, row2);
            } else {
                wave_batched<G>(list, wk, q, pre, row);
            }
        };
        if (CL != NCLS) body(std::integral_constant<int, GS>{}, std::integral_constant<int, RS>{}, CL, blockIdx.x, nblk);
        else if ((int)blockIdx.x < a.gS)
            body(std::integral_constant<int, GS>{}, std::integral_constant<int, RS>{}, CLS_S, blockIdx.x, a.gS);
        else
            body(std::integral_constant<int, 8>{}, std::integral_constant<int, 8>{}, CLS_S2, blockIdx.x - a.gS, a.gS2);
    } else if (ROLE == 2) {
        // one wave per row; lanes first inspect a stretch of the class list at
        // once (part, lock stamp and row bounds of up to 64 vertices in one
        // round trip) and queue the rows that need work
        const int ng = BLOCK / 64;
        for (int i = threadIdx.x; i < ng * stride; i += BLOCK) lds[i] = 0;
        __syncthreads();
        int32_t *tab = lds + (threadIdx.x >> 6) * stride;
        int32_t *q = lds + ng * stride + (threadIdx.x >> 6) * 64;
        const int wid = blockIdx.x * ng + (threadIdx.x >> 6), nwaves = nblk * ng;
        const bool scan = a.k <= WAVE_SCAN_KMAX;
        for (int c = 1; c < NCLS; c++) {
            if (a.tmap[c] != 2) continue;
            const int cnt = a.binoff[c + 1] - a.binoff[c];
            const int unit = wave_unit(cnt, nwaves);
            auto pre = [&](Meta &m) -> bool {
                m.g = gof<B>(a, m.v);
                pv.sel<B>(a, m.g);
                if (pv.kind != KIND_LP) return false;
                m.ps = a.P[m.v];
                const int lk = a.lock[m.v];
                const int64_t x0 = a.xadj[m.v], x1 = a.xadj[m.v + 1];
                pacc.sel<B>(a, m.g);
                pacc.c0++;
                if (lk == pv.lp_id - 1) {
                    gain_locked(a, m.v, m.ps);
                    return false;
                }
                m.s = x0;
                m.deg = (int)(x1 - x0);
                pacc.c1++;
                pacc.c2 += m.deg;
                return true;
            };
            auto row = [&](const Meta &t, int gl) {
                rv.sel<B>(a, t.g);
                uint64_t best = 0;
                int cs = 0;
                if (scan) {
                    group_fill_row<64, 16>(a, t.s, t.deg, gl, tab);
                    for (int p = gl; p < rv.k; p += 64) {
                        const int cc = tab[p];
                        if (cc) {
                            tab[p] = 0;
                            if (p == t.ps) cs = cc;
                            else {
                                const uint64_t k2 = conn_key(cc, p);
                                best = k2 > best ? k2 : best;
                            }
                        }
                    }
                    lds_fence_wave();
                } else {
                    int pu[16], cu[16];
                    group_conn_row<64, 16>(a, t.s, t.deg, gl, tab, pu, cu);
#pragma unroll
                    for (int r = 0; r < 16; r++) {
                        if (cu[r] > 0) {
                            if (pu[r] == t.ps) cs += cu[r];
                            else {
                                const uint64_t k2 = conn_key(cu[r], pu[r]);
                                best = k2 > best ? k2 : best;
                            }
                        }
                    }
                }
                best = gmax_u64<64>(best);
                cs = gsum<64>(cs);
                if (gl == 0) {
                    racc.sel<B>(a, t.g);
                    racc.c0 += gain_finish(a, t.v, t.ps, best, cs, rv.cn, rv.cd);
                }
            };
            wave_batched<64>(a.bins + a.binoff[c], walk_q<B>(a, cnt, wid, nwaves, unit, WQ_GAIN2 + c), q, pre, row,
                             unit);
        }
    } else {
        for (int i = threadIdx.x; i < a.k; i += BLOCK) lds[i] = 0;
        __syncthreads();
        for (int c = 1; c < NCLS; c++)
            if (a.tmap[c] == 3) gain_blocks<B>(a, c, lds, blockIdx.x, nblk, pv, pacc, racc);
    }
    acc_finish(a, pacc);
    acc_finish(a, racc);
}

template <bool B, int ROLE, int GS = 8, int RS = 32 / GS, int CL = CLS_S>
__global__ __launch_bounds__(BLOCK) void k_gain(KArgs a, int nblk)
{
    if (!any_kind(a, KIND_LP)) return;
    // one graph's small class alone (the finest levels of a mesh): its own
    // launch, so the paired rows get their register budget
    gain_body<B, ROLE, GS, RS, CL, !B && ROLE == 1 && CL == CLS_S>(a, nblk);
}

// -------------------------------------------------------------- afterburner --

// F2(v) = sum over neighbours u of w * ([q_u = P_d(v)] - [q_u = P_s(v)]) with
// q_u = P_d(u) when u is in X and precedes v (larger F, or equal F and smaller
// id), else P_s(u). Moves with F2 >= 0 form M.
template <int U, bool NT = false>
__device__ __forceinline__ int after_sum_row(const KArgs &a, int v, int64_t s, int deg, int ps, int pd, int Fv, int gl,
                                             int stride)
{
    int sum = 0;
    if (a.rq) {
        // one 4-byte gather per neighbour (parts and saturated F)
        for (int base = gl; base < deg; base += stride * U) {
            int u[U], wt[U];
            uint32_t q[U];
#pragma unroll
            for (int j = 0; j < U; j++) {
                const int idx = base + j * stride;
                u[j] = idx < deg ? ld_adj<NT>(a, s + idx) : -1;
                wt[j] = idx < deg ? ld_ew<NT>(a, s + idx) : 0;
            }
#pragma unroll
            for (int j = 0; j < U; j++) q[j] = u[j] >= 0 ? ((const uint32_t *)a.rq)[u[j]] : 0u;
#pragma unroll
            for (int j = 0; j < U; j++) {
                if (u[j] < 0) continue;
                int qp = (int)(q[j] >> 24);
                const int pqu = (int)((q[j] >> 16) & 0xFFu);
                if (pqu != qp) {
                    int Fu = (int)(int16_t)(q[j] & 0xFFFFu);
                    if ((Fu == 32767 && Fv >= 32767) || (Fu == -32768 && Fv <= -32768)) Fu = a.Fx[u[j]];
                    if (Fu > Fv || (Fu == Fv && u[j] < v)) qp = pqu;
                }
                sum += qp == pd ? wt[j] : (qp == ps ? -wt[j] : 0);
            }
        }
        return sum;
    }
    for (int base = gl; base < deg; base += stride * U) {
        int u[U], wt[U];
        int2 ru[U];
#pragma unroll
        for (int j = 0; j < U; j++) {
            const int idx = base + j * stride;
            u[j] = idx < deg ? ld_adj<NT>(a, s + idx) : -1;
            wt[j] = idx < deg ? ld_ew<NT>(a, s + idx) : 0;
        }
#pragma unroll
        for (int j = 0; j < U; j++) ru[j] = u[j] >= 0 ? a.rec[u[j]] : make_int2(0, 0);
#pragma unroll
        for (int j = 0; j < U; j++) {
            if (u[j] < 0) continue;
            int q = ru[j].x >> 16;
            const int pdu = (ru[j].x & 0xFFFF) - 1;
            if (pdu >= 0 && (ru[j].y > Fv || (ru[j].y == Fv && u[j] < v))) q = pdu;
            sum += q == pd ? wt[j] : (q == ps ? -wt[j] : 0);
        }
    }
    return sum;
}

// rx: the vertex's record word (P_s << 16 | P_d + 1).
__device__ __forceinline__ void after_store(const KArgs &a, int v, int rx, int sum)
{
    if (a.dbg_F2) a.dbg_F2[v] = sum;
    if (sum >= 0) {
        const int pd = (rx & 0xFFFF) - 1;
        a.dest[v] = pd;
        mq_set(a, v, rx >> 16, pd);
    }
}

// Jetlp ablation without the afterburner: every vertex of X moves.
__device__ __forceinline__ bool no_afterburner(const KArgs &a, int g)
{
    return a.ctl[g].flags & JET_F_LP_NO_AFTERBURNER;
}

template <bool B>
__device__ void afterburner_body(const KArgs &a, int b)
{
    __shared__ int32_t s_red[BLOCK / 64];
    __shared__ int32_t s_q[BLOCK];
    if (!any_kind(a, KIND_LP)) return;
    GV pv;
    if (!B) pv.at(a, 0);
    if (b < a.gS) {
        int32_t *q = s_q + (threadIdx.x >> 6) * 64;
        wave_batched<8>(
            (!B && a.sident) ? nullptr : a.bins + a.binoff[CLS_S],
            walk_q<B>(a, a.binoff[CLS_S2 + 1] - a.binoff[CLS_S], b * (BLOCK / 64) + (threadIdx.x >> 6),
                      a.gS * (BLOCK / 64), 64, WQ_AFTER_S),
            q,
            [&](Meta &m) -> bool {
                const int g = gof<B>(a, m.v);
                pv.sel<B>(a, g);
                if (pv.kind != KIND_LP) return false;
                const int2 r = own_rec(a, m.v);
                if ((r.x & 0xFFFF) == 0) return false;  // not in X
                if (no_afterburner(a, g)) {
                    after_store(a, m.v, r.x, 0);
                    return false;
                }
                m.ps = r.x;
                m.aux = r.y;
                m.s = a.xadj[m.v];
                m.deg = (int)(a.xadj[m.v + 1] - m.s);
                return true;
            },
            [&](const Meta &t, int gl) {
                const int ps = t.ps >> 16, pd = (t.ps & 0xFFFF) - 1;
                int sum = after_sum_row<4>(a, t.v, t.s, t.deg, ps, pd, t.aux, gl, 8);
                sum = gsum<8>(sum);
                if (gl == 0) after_store(a, t.v, t.ps, sum);
            });
        return;
    }
    b -= a.gS;
    if (b < a.gM) {
        // one wave per row of X; lanes first inspect a stretch of the list at once
        int32_t *q = s_q + (threadIdx.x >> 6) * 64;
        const int cnt = a.binoff[CLS_M + 1] - a.binoff[CLS_M], nw = a.gM * (BLOCK / 64);
        const int unit = wave_unit(cnt, nw);
        wave_batched<64>(
            a.bins + a.binoff[CLS_M], walk_q<B>(a, cnt, b * (BLOCK / 64) + (threadIdx.x >> 6), nw, unit, WQ_AFTER_M), q,
            [&](Meta &m) -> bool {
                const int g = gof<B>(a, m.v);
                pv.sel<B>(a, g);
                if (pv.kind != KIND_LP) return false;
                const int2 r = own_rec(a, m.v);
                if ((r.x & 0xFFFF) == 0) return false;  // not in X
                if (no_afterburner(a, g)) {
                    after_store(a, m.v, r.x, 0);
                    return false;
                }
                m.ps = r.x;
                m.aux = r.y;
                m.s = a.xadj[m.v];
                m.deg = (int)(a.xadj[m.v + 1] - m.s);
                return true;
            },
            [&](const Meta &t, int gl) {
                const int ps = t.ps >> 16, pd = (t.ps & 0xFFFF) - 1;
                int sum = after_sum_row<4, true>(a, t.v, t.s, t.deg, ps, pd, t.aux, gl, 64);
                sum = gsum<64>(sum);
                if (gl == 0) after_store(a, t.v, t.ps, sum);
            },
            unit);
        return;
    }
    b -= a.gM;
    if (b >= a.gL) return;
    const int32_t *list = a.bins + a.binoff[CLS_L];
    const Walk w = walk<B>(a.binoff[CLS_L + 1] - a.binoff[CLS_L], b, a.gL, 1);
    for (int i = w.first; i < w.end; i += w.step) {
        const int v = list[i];
        const int g = gof<B>(a, v);
        pv.sel<B>(a, g);
        if (pv.kind != KIND_LP) continue;
        const int2 r = own_rec(a, v);
        if ((r.x & 0xFFFF) == 0) continue;
        const int ps = r.x >> 16, pd = (r.x & 0xFFFF) - 1;
        if (no_afterburner(a, g)) {
            if (threadIdx.x == 0) after_store(a, v, r.x, 0);
            continue;
        }
        const int64_t s = a.xadj[v];
        int sum = after_sum_row<UROW, true>(a, v, s, (int)(a.xadj[v + 1] - s), ps, pd, r.y, threadIdx.x, BLOCK);
        sum = block_sum<BLOCK>(sum, s_red);
        if (threadIdx.x == 0) after_store(a, v, r.x, sum);
    }
}

// ------------------------------------------------- cut change of the moves --

// Delta of the cut over the edges of moved vertices: an edge whose two ends
// both move is counted from its smaller end. Moved count, weight and digest
// change are counted by the lane that finds the move.
template <int U, bool NT = false>
__device__ __forceinline__ int dcut_sum_row(const KArgs &a, int v, int64_t s, int deg, int ps, int pn, int gl,
                                            int stride)
{
    int delta = 0;
    const int sh = a.P8 ? 8 : 16;
    const uint32_t lo = a.P8 ? 0xFFu : 0xFFFFu;
    for (int base = gl; base < deg; base += stride * U) {
        int u[U], wt[U];
        uint32_t q[U];
#pragma unroll
        for (int j = 0; j < U; j++) {
            const int idx = base + j * stride;
            u[j] = idx < deg ? ld_adj<NT>(a, s + idx) : -1;
            wt[j] = idx < deg ? ld_ew<NT>(a, s + idx) : 0;
        }
#pragma unroll
        for (int j = 0; j < U; j++) q[j] = u[j] >= 0 ? mq_load(a, u[j]) : 0u;
#pragma unroll
        for (int j = 0; j < U; j++) {
            // a neighbour that moves too (new part != old part) and has the
            // smaller id counts the edge from its own row
            const int pu = (int)(q[j] >> sh), pun = (int)(q[j] & lo);
            if (u[j] < 0 || (pun != pu && u[j] < v)) continue;
            delta += wt[j] * ((int)(pn != pun) - (int)(ps != pu));
        }
    }
    return delta;
}

typedef GAcc<ST_M, ST_MW, ST_DIG> MoveAcc;
typedef GAcc<ST_DCUT> CutAcc;

__device__ __forceinline__ void move_meta(const KArgs &a, int v, int lv, int ps, int pn, MoveAcc &acc)
{
    acc.c0++;
    acc.c1 += a.vw ? a.vw[v] : 1;
    acc.c2 += mix64(((uint64_t)(uint32_t)lv << 32) | (uint32_t)pn) - mix64(((uint64_t)(uint32_t)lv << 32) | (uint32_t)ps);
}

template <bool B>
__global__ __launch_bounds__(BLOCK) void k_dcut(KArgs a)
{
    __shared__ int32_t s_red32[BLOCK / 64];
    __shared__ int32_t s_q[BLOCK];
    if (!any_active(a)) return;
    GV pv;
    if (!B) pv.at(a, 0);
    if (count_row(a)[0] > 0) {
        // graphs whose previous iteration improved the best partition: copy
        // P_iter before this iteration's moves are applied
        int lo, hi;
        flat_range<B>(a, lo, hi);
        for (int i = lo + threadIdx.x; i < hi; i += BLOCK) {
            const int v = flat_vertex<B>(a, i);
            pv.sel<B>(a, gof<B>(a, v));
            if (pv.copy && pv.kind != KIND_DONE) a.best[v] = a.P[v];
        }
    }
    MoveAcc macc;
    CutAcc cacc;
    if (!B) {
        macc.to(a, 0);
        cacc.to(a, 0);
    }
    int b = blockIdx.x;
    if (b < a.gS) {
        int32_t *q = s_q + (threadIdx.x >> 6) * 64;
        wave_batched<8>(
            (!B && a.sident) ? nullptr : a.bins + a.binoff[CLS_S],
            walk_q<B>(a, a.binoff[CLS_S2 + 1] - a.binoff[CLS_S], b * (BLOCK / 64) + (threadIdx.x >> 6),
                      a.gS * (BLOCK / 64), 64, WQ_DCUT_S),
            q,
            [&](Meta &m) -> bool {
                const int pn = a.dest[m.v];
                if (pn < 0) return false;
                m.aux = pn;
                m.ps = a.P[m.v];
                m.g = gof<B>(a, m.v);
                pv.sel<B>(a, m.g);
                macc.sel<B>(a, m.g);
                move_meta(a, m.v, m.v - pv.voff, m.ps, pn, macc);
                m.s = a.xadj[m.v];
                m.deg = (int)(a.xadj[m.v + 1] - m.s);
                return true;
            },
            [&](const Meta &t, int gl) {
                int d = dcut_sum_row<4>(a, t.v, t.s, t.deg, t.ps, t.aux, gl, 8);
                d = gsum<8>(d);
                if (gl == 0) {
                    cacc.sel<B>(a, t.g);
                    cacc.c0 += (uint64_t)(int64_t)d;
                }
            });
    } else if ((b -= a.gS) < a.gM) {
        // one wave per moved row; lanes first inspect a stretch of the list at once
        int32_t *q = s_q + (threadIdx.x >> 6) * 64;
        const int cnt = a.binoff[CLS_M + 1] - a.binoff[CLS_M], nw = a.gM * (BLOCK / 64);
        const int unit = wave_unit(cnt, nw);
        wave_batched<64>(
            a.bins + a.binoff[CLS_M], walk_q<B>(a, cnt, b * (BLOCK / 64) + (threadIdx.x >> 6), nw, unit, WQ_DCUT_M), q,
            [&](Meta &m) -> bool {
                const int pn = a.dest[m.v];
                if (pn < 0) return false;
                m.aux = pn;
                m.ps = a.P[m.v];
                m.g = gof<B>(a, m.v);
                pv.sel<B>(a, m.g);
                macc.sel<B>(a, m.g);
                move_meta(a, m.v, m.v - pv.voff, m.ps, pn, macc);
                m.s = a.xadj[m.v];
                m.deg = (int)(a.xadj[m.v + 1] - m.s);
                return true;
            },
            [&](const Meta &t, int gl) {
                int d = dcut_sum_row<4, true>(a, t.v, t.s, t.deg, t.ps, t.aux, gl, 64);
                d = gsum<64>(d);
                if (gl == 0) {
                    cacc.sel<B>(a, t.g);
                    cacc.c0 += (uint64_t)(int64_t)d;
                }
            },
            unit);
    } else if ((b -= a.gM) < a.gL) {
        const int32_t *list = a.bins + a.binoff[CLS_L];
        const Walk w = walk<B>(a.binoff[CLS_L + 1] - a.binoff[CLS_L], b, a.gL, 1);
        for (int i = w.first; i < w.end; i += w.step) {
            const int v = list[i];
            const int pn = a.dest[v];
            if (pn < 0) continue;
            const int ps = a.P[v];
            const int g = gof<B>(a, v);
            const int64_t s = a.xadj[v];
            int d = dcut_sum_row<UROW, true>(a, v, s, (int)(a.xadj[v + 1] - s), ps, pn, threadIdx.x, BLOCK);
            d = block_sum<BLOCK>(d, s_red32);
            if (threadIdx.x == 0) {
                pv.sel<B>(a, g);
                macc.sel<B>(a, g);
                move_meta(a, v, v - pv.voff, ps, pn, macc);
                cacc.sel<B>(a, g);
                cacc.c0 += (uint64_t)(int64_t)d;
            }
        }
    } else if ((b -= a.gL) < a.gZ) {
        const int32_t *list = a.bins + a.binoff[CLS_Z];
        const int cnt = a.binoff[CLS_Z + 1] - a.binoff[CLS_Z];
        int lo, hi;
        block_chunk(cnt, b, a.gZ, lo, hi);
        for (int i = lo + threadIdx.x; i < hi; i += BLOCK) {
            const int v = list[i];
            const int pn = a.dest[v];
            if (pn < 0) continue;
            const int g = gof<B>(a, v);
            pv.sel<B>(a, g);
            macc.sel<B>(a, g);
            move_meta(a, v, v - pv.voff, a.P[v], pn, macc);
        }
    }
    acc_finish(a, macc);
    acc_finish(a, cacc);
}

// ------------------------------------------------------------ apply moves --

template <bool B>
__global__ __launch_bounds__(BLOCK) void k_apply(KArgs a)
{
    extern __shared__ int32_t s_dw[];  // [k] block-partial weight change (one graph)
    if (!any_active(a)) return;
    constexpr bool single = !B;
    if (single) {
        for (int p = threadIdx.x; p < a.k; p += BLOCK) s_dw[p] = 0;
        __syncthreads();
    }
    GV pv;
    if (!B) pv.at(a, 0);
    int lo, hi;
    flat_range<B>(a, lo, hi);
    for (int i = lo + threadIdx.x; i < hi; i += BLOCK) {
        const int v = flat_vertex<B>(a, i);
        const int pn = a.dest[v];
        if (pn < 0) continue;
        pv.sel<B>(a, gof<B>(a, v));
        const int ps = a.P[v];
        const int vwv = a.vw ? a.vw[v] : 1;
        a.P[v] = (uint16_t)pn;
        if (a.P8) a.P8[v] = (uint8_t)pn;
        mq_set(a, v, pn, pn);
        a.dest[v] = -1;
        if (pv.kind == KIND_LP) a.lock[v] = pv.lp_id;
        if (single) {
            atomicSub(&s_dw[ps], vwv);
            atomicAdd(&s_dw[pn], vwv);
        } else {
            atomicAdd((unsigned long long *)&a.w[pv.poff + ps], (unsigned long long)(-(int64_t)vwv));
            atomicAdd((unsigned long long *)&a.w[pv.poff + pn], (unsigned long long)(int64_t)vwv);
        }
    }
    if (single) {
        __syncthreads();
        for (int p = threadIdx.x; p < a.k; p += BLOCK)
            if (s_dw[p]) atomicAdd((unsigned long long *)&a.w[p], (unsigned long long)(int64_t)s_dw[p]);
    }
}

// Candidate test without side effects (the chunked rows write the
// "no candidate" outputs once, from the vertex's first chunk).
__device__ __forceinline__ bool rb_is_candidate(const KArgs &a, int ps, int vwv, const GV &gv)
{
    const int gp = gv.poff + ps;
    const int64_t k = gv.k;
    return a.isA[gp] && 2 * k * vwv <= 3 * (k * a.w[gp] - gv.W);
}

// ------------------------------------------------------- chunked long rows --
// Rows of the L class (more than M_MAXDEG entries) are cut into chunks of
// LCHUNK entries, one block each (16 entries per thread, every load of the
// chunk issued before its gathers), spread over the whole grid. A connectivity
// pass adds a chunk's part counts into a block-shared LDS table. A row of one
// chunk finishes in that block, as the block role would. A longer row stores
// each chunk's table in a global row of its own (plain coalesced stores, no
// atomics: chunks of one hub no longer meet on the same addresses), and a
// second kernel (one wave per such vertex) sums the rows of its chunks and
// finishes it. The afterburner and cut-delta passes reduce a chunk's partial
// sum over the block. Kernel boundaries order the phases.
constexpr int LCHUNK = BLOCK * 16;

enum HistMode { HIST_NONE = 0, HIST_LDS = 1, HIST_GLOBAL = 2 };
__device__ __forceinline__ void rb_finish(const KArgs &a, int v, int ps, const GV &gv, uint64_t best, int cs, int sumB,
                                          int cntB, int vwv, int hmode, int32_t *lh);

struct LChunk {
    int v, li, len;
    bool multi;  // the row has more than one chunk
    int64_t s;
};

__device__ __forceinline__ LChunk lchunk(const KArgs &a, int i)
{
    const int2 e = a.lch[i];
    LChunk ch;
    ch.li = e.x;
    ch.v = a.bins[a.binoff[CLS_L] + e.x];
    const int64_t s = a.xadj[ch.v], deg = a.xadj[ch.v + 1] - s;
    ch.s = s + (int64_t)e.y * LCHUNK;
    const int64_t rest = deg - (int64_t)e.y * LCHUNK;
    ch.len = (int)(rest < LCHUNK ? rest : LCHUNK);
    ch.multi = deg > LCHUNK;
    return ch;
}

// The whole block adds the part counts of a chunk (len <= LCHUNK entries)
// into `tab`.
__device__ __forceinline__ void chunk_fill(const KArgs &a, int64_t s, int len, int32_t *tab)
{
    constexpr int U = LCHUNK / BLOCK;
    int u[U], w[U];
#pragma unroll
    for (int j = 0; j < U; j++) {
        const int idx = threadIdx.x + j * BLOCK;
        u[j] = idx < len ? ld_adj<true>(a, s + idx) : -1;
        w[j] = idx < len ? ld_ew<true>(a, s + idx) : 0;
    }
#pragma unroll
    for (int j = 0; j < U; j++) u[j] = u[j] >= 0 ? gpart(a, u[j]) : -1;
#pragma unroll
    for (int j = 0; j < U; j++)
        if (u[j] >= 0) atomicAdd(&tab[u[j]], w[j]);
    __syncthreads();
}

// Moves a chunk's table to its global row (every part, zeros included, so
// the finishing kernel needs no clearing) and clears the table.
__device__ __forceinline__ void chunk_store(const KArgs &a, int i, int k, int32_t *tab)
{
    int32_t *row = a.gconn + (int64_t)i * a.lstride;
    for (int p = threadIdx.x; p < k; p += BLOCK) {
        const int c = tab[p];
        row[p] = c;
        if (c) tab[p] = 0;
    }
    __syncthreads();
}

// Jetlp gain (RB = false) or rebalancing loss (RB = true) of the long rows,
// first phase: one block per chunk.
template <bool B, bool RB>
__global__ __launch_bounds__(BLOCK) void k_lconn(KArgs a, int hmode)
{
    __shared__ uint64_t s_red[BLOCK / 64];
    __shared__ int32_t s_red32[BLOCK / 64];
    if (RB ? !any_rb(a) : !any_kind(a, KIND_LP)) return;
    extern __shared__ int32_t lds[];
    for (int i = threadIdx.x; i < a.k; i += BLOCK) lds[i] = 0;
    __syncthreads();
    GV pv;
    GainPre pacc;
    CountX racc;
    if (!B) {
        pv.at(a, 0);
        pacc.to(a, 0);
        racc.to(a, 0);
    }
    for (int i = blockIdx.x; i < a.nlch; i += gridDim.x) {
        const LChunk ch = lchunk(a, i);
        const int g = gof<B>(a, ch.v);
        pv.sel<B>(a, g);
        const int ps = a.P[ch.v];
        const int vwv = a.vw ? a.vw[ch.v] : 1;
        if (RB) {
            if (!is_rb(pv.kind) || !rb_is_candidate(a, ps, vwv, pv)) continue;
        } else {
            if (pv.kind != KIND_LP || a.lock[ch.v] == pv.lp_id - 1) continue;
        }
        chunk_fill(a, ch.s, ch.len, lds);
        if (ch.multi) {
            chunk_store(a, i, pv.k, lds);
            continue;
        }
        // a row of one chunk: finish the vertex here
        uint64_t best = 0;
        int cs = 0, sumB = 0, cntB = 0;
        for (int p = threadIdx.x; p < pv.k; p += BLOCK) {
            const int c = lds[p];
            if (c) {
                lds[p] = 0;
                if (p == ps) cs = c;
                else if (!RB || a.isB[pv.poff + p]) {
                    const uint64_t k2 = conn_key(c, p);
                    best = k2 > best ? k2 : best;
                    sumB += c;
                    cntB++;
                }
            }
        }
        best = block_max_u64<BLOCK>(best, s_red);
        cs = block_sum<BLOCK>(cs, s_red32);
        if (RB) {
            sumB = block_sum<BLOCK>(sumB, s_red32);
            cntB = block_sum<BLOCK>(cntB, s_red32);
        }
        if (threadIdx.x == 0) {
            racc.sel<B>(a, g);
            if (RB) {
                rb_finish(a, ch.v, ps, pv, best, cs, sumB, cntB, vwv, hmode, nullptr);
                racc.c0++;
            } else {
                pacc.sel<B>(a, g);
                pacc.c0++;
                pacc.c1++;
                pacc.c2 += ch.len;
                racc.c0 += gain_finish(a, ch.v, ps, best, cs, pv.cn, pv.cd);
            }
        }
    }
    if (!RB) acc_finish(a, pacc);
    acc_finish(a, racc);
}

// Sum of a multi-chunk row's chunk tables at part p.
__device__ __forceinline__ int chunk_rows_sum(const KArgs &a, int li, int p)
{
    const int c0 = a.lcoff[li], c1 = a.lcoff[li + 1];
    int c = 0;
    for (int i = c0; i < c1; i++) c += a.gconn[(int64_t)i * a.lstride + p];
    return c;
}

// Phase 2 of the Jetlp gain on long rows (one wave per vertex): locked rows,
// and the rows of more than one chunk.
template <bool B>
__global__ __launch_bounds__(BLOCK) void k_lgain_fin(KArgs a)
{
    if (!any_kind(a, KIND_LP)) return;
    const int gl = threadIdx.x & 63;
    const int nL = a.binoff[CLS_L + 1] - a.binoff[CLS_L];
    GV pv;
    GainPre pacc;
    CountX racc;
    if (!B) {
        pv.at(a, 0);
        pacc.to(a, 0);
        racc.to(a, 0);
    }
    const int nw = gridDim.x * (BLOCK / 64);
    for (int li = blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6); li < nL; li += nw) {
        const int v = a.bins[a.binoff[CLS_L] + li];
        const int g = gof<B>(a, v);
        pv.sel<B>(a, g);
        if (pv.kind != KIND_LP) continue;
        const int ps = a.P[v];
        if (a.lock[v] == pv.lp_id - 1) {
            if (gl == 0) {
                pacc.sel<B>(a, g);
                pacc.c0++;
                gain_locked(a, v, ps);
            }
            continue;
        }
        const int64_t deg = a.xadj[v + 1] - a.xadj[v];
        if (deg <= LCHUNK) continue;  // finished by its chunk's block
        uint64_t best = 0;
        int cs = 0;
        for (int p = gl; p < pv.k; p += 64) {
            const int c = chunk_rows_sum(a, li, p);
            if (c) {
                if (p == ps) cs = c;
                else {
                    const uint64_t k2 = conn_key(c, p);
                    best = k2 > best ? k2 : best;
                }
            }
        }
        best = gmax_u64<64>(best);
        cs = gsum<64>(cs);
        if (gl == 0) {
            pacc.sel<B>(a, g);
            pacc.c0++;
            pacc.c1++;
            pacc.c2 += deg;
            racc.sel<B>(a, g);
            racc.c0 += gain_finish(a, v, ps, best, cs, pv.cn, pv.cd);
        }
    }
    acc_finish(a, pacc);
    acc_finish(a, racc);
}

// Afterburner on long rows, phase 1: the F2 sum of every chunk of a vertex
// in X; a row of one chunk stores its move here.
template <bool B>
__global__ __launch_bounds__(BLOCK) void k_lafter(KArgs a)
{
    __shared__ int32_t s_red[BLOCK / 64];
    if (!any_kind(a, KIND_LP)) return;
    GV pv;
    if (!B) pv.at(a, 0);
    for (int i = blockIdx.x; i < a.nlch; i += gridDim.x) {
        const LChunk ch = lchunk(a, i);
        const int g = gof<B>(a, ch.v);
        pv.sel<B>(a, g);
        if (pv.kind != KIND_LP || no_afterburner(a, g)) continue;
        const int2 r = own_rec(a, ch.v);
        if ((r.x & 0xFFFF) == 0) continue;  // not in X
        const int ps = r.x >> 16, pd = (r.x & 0xFFFF) - 1;
        int part = after_sum_row<8, true>(a, ch.v, ch.s, ch.len, ps, pd, r.y, threadIdx.x, BLOCK);
        part = block_sum<BLOCK>(part, s_red);
        if (threadIdx.x == 0) {
            if (!ch.multi) after_store(a, ch.v, r.x, part);
            else if (part) atomicAdd(&a.gf2[ch.li], part);
        }
    }
}

// Afterburner on long rows, phase 2 (one lane per vertex): rows of more than
// one chunk, and the ablation without the afterburner.
template <bool B>
__global__ __launch_bounds__(BLOCK) void k_lafter_fin(KArgs a)
{
    if (!any_kind(a, KIND_LP)) return;
    const int nL = a.binoff[CLS_L + 1] - a.binoff[CLS_L];
    GV pv;
    if (!B) pv.at(a, 0);
    for (int li = blockIdx.x * BLOCK + threadIdx.x; li < nL; li += gridDim.x * BLOCK) {
        const int v = a.bins[a.binoff[CLS_L] + li];
        const int g = gof<B>(a, v);
        pv.sel<B>(a, g);
        if (pv.kind != KIND_LP) continue;
        const int2 r = own_rec(a, v);
        if ((r.x & 0xFFFF) == 0) continue;
        if (no_afterburner(a, g)) {
            after_store(a, v, r.x, 0);
            continue;
        }
        if (a.xadj[v + 1] - a.xadj[v] <= LCHUNK) continue;
        const int sum = a.gf2[li];
        a.gf2[li] = 0;
        after_store(a, v, r.x, sum);
    }
}

template <bool B>
__global__ __launch_bounds__(BLOCK) void k_ldcut(KArgs a)
{
    __shared__ int32_t s_red[BLOCK / 64];
    if (!any_active(a)) return;
    GV pv;
    MoveAcc macc;
    CutAcc cacc;
    if (!B) {
        pv.at(a, 0);
        macc.to(a, 0);
        cacc.to(a, 0);
    }
    for (int i = blockIdx.x; i < a.nlch; i += gridDim.x) {
        const LChunk ch = lchunk(a, i);
        const int pn = a.dest[ch.v];
        if (pn < 0) continue;
        const int ps = a.P[ch.v];
        int d = dcut_sum_row<8, true>(a, ch.v, ch.s, ch.len, ps, pn, threadIdx.x, BLOCK);
        d = block_sum<BLOCK>(d, s_red);
        if (threadIdx.x == 0) {
            const int g = gof<B>(a, ch.v);
            cacc.sel<B>(a, g);
            cacc.c0 += (uint64_t)(int64_t)d;
            if (a.lch[i].y == 0) {
                pv.sel<B>(a, g);
                macc.sel<B>(a, g);
                move_meta(a, ch.v, ch.v - pv.voff, ps, pn, macc);
            }
        }
    }
    acc_finish(a, macc);
    acc_finish(a, cacc);
}

// Set-up of the chunk list: chunks per L vertex, their exclusive scan (total
// in lmeta[0]) and the list itself. ctot holds the class totals.
__global__ __launch_bounds__(BLOCK) void k_lchunk_count(const int64_t *xadj, const int32_t *bins, const int32_t *ctot,
                                                        int32_t *lcnt)
{
    const int off = ctot[CLS_Z] + ctot[CLS_S] + ctot[CLS_S2] + ctot[CLS_M], nL = ctot[CLS_L];
    for (int li = blockIdx.x * BLOCK + threadIdx.x; li < nL; li += gridDim.x * BLOCK) {
        const int v = bins[off + li];
        lcnt[li] = (int)((xadj[v + 1] - xadj[v] + LCHUNK - 1) / LCHUNK);
    }
}

__global__ __launch_bounds__(BLOCK) void k_lchunk_scan(const int32_t *ctot, int32_t *lcnt, int32_t *lmeta)
{
    __shared__ int32_t s_scan[BLOCK / 64];
    const int nL = ctot[CLS_L];
    int32_t carry = 0;
    for (int b0 = 0; b0 < nL; b0 += BLOCK) {
        const int i = b0 + threadIdx.x;
        const int32_t x = i < nL ? lcnt[i] : 0;
        int32_t tot;
        const int32_t ex = block_excl_scan<BLOCK>(x, s_scan, tot);
        if (i < nL) lcnt[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        lcnt[nL] = carry;
        lmeta[0] = carry;
    }
}

__global__ __launch_bounds__(BLOCK) void k_lchunk_fill(const int32_t *ctot, const int32_t *lcoff, int2 *lch)
{
    const int nL = ctot[CLS_L];
    for (int li = blockIdx.x * BLOCK + threadIdx.x; li < nL; li += gridDim.x * BLOCK)
        for (int c = 0; c < lcoff[li + 1] - lcoff[li]; c++) lch[lcoff[li] + c] = make_int2(li, c);
}

// -------------------------------------------------------------- rebalance --

// Loss of an eligible vertex of an oversized part (Jetrw: own connectivity
// minus that of the best connected valid destination, ties -> smaller id, or
// a random valid destination when none is adjacent; Jetrs: own connectivity
// minus the floor mean over adjacent valid destinations) and its slot.
// Histogram of the candidates' (part, slot) weights, when the loss kernels
// build it: HIST_LDS adds into the block's LDS copy (flushed once per block),
// HIST_GLOBAL adds into the global histogram directly; HIST_NONE leaves it to
// the separate histogram pass.
__device__ __forceinline__ void rb_finish(const KArgs &a, int v, int ps, const GV &gv, uint64_t best, int cs, int sumB,
                                          int cntB, int vwv, int hmode, int32_t *lh)
{
    int loss, d = -1;
    if (gv.kind == KIND_RW) {
        if (best) {
            d = (int)(~(uint32_t)best);
            loss = cs - (int)(best >> 32);
        } else if (gv.nB > 0) {
            const uint64_t h = mix64(gv.hs ^ (uint64_t)(uint32_t)(v - gv.voff));
            d = a.Blist[gv.poff + (int)__umul64hi(h, (uint64_t)gv.nB)];
            loss = cs;
        } else {
            d = ps;  // unreachable: the lightest part is always a valid destination
            loss = cs;
        }
        a.rbd[v] = d;
    } else {
        loss = cs - (cntB ? sumB / cntB : 0);
    }
    const int s = loss_slot(loss);
    a.slot[v] = (uint8_t)s;
    if (hmode == HIST_LDS) atomicAdd(&lh[ps * NSLOT + s], vwv);
    else if (hmode == HIST_GLOBAL)
        atomicAdd((unsigned long long *)&a.hist[(int64_t)(gv.poff + ps) * NSLOT + s], (unsigned long long)(int64_t)vwv);
    if (a.dbg_loss) {
        a.dbg_loss[v] = loss;
        a.dbg_slot[v] = s;
        a.dbg_pd[v] = d;
    }
}

// Outputs of a vertex that is no rebalancing candidate.
__device__ __forceinline__ void rb_no_candidate(const KArgs &a, int v)
{
    a.slot[v] = 255;
    if (a.dbg_loss) {
        a.dbg_loss[v] = INT64_MIN;
        a.dbg_slot[v] = -1;
        a.dbg_pd[v] = -1;
    }
}

// Candidate test: the vertex's part is oversized and its weight is small
// enough (2k * vw <= 3 (k * w(P_s) - W)). Writes the "no candidate" outputs.
__device__ __forceinline__ bool rb_candidate(const KArgs &a, int v, int ps, int vwv, const GV &gv)
{
    if (rb_is_candidate(a, ps, vwv, gv)) return true;
    rb_no_candidate(a, v);
    return false;
}

template <bool B, int G, int R>
__device__ void rb_groups(const KArgs &a, int cls, int32_t *tab, int gid, int ngroups, GV &gv, CountX &racc, int hmode,
                          int32_t *lh)
{
    const int gl = threadIdx.x & (G - 1);
    const int32_t *list = a.bins + a.binoff[cls];
    const Walk w = walk<B>(a.binoff[cls + 1] - a.binoff[cls], gid, ngroups, 1);
    for (int i = w.first; i < w.end; i += w.step) {
        const int v = list[i];
        const int g = gof<B>(a, v);
        gv.sel<B>(a, g);
        if (!is_rb(gv.kind)) continue;
        const int ps = a.P[v];
        const int vwv = a.vw ? a.vw[v] : 1;
        if (!rb_candidate(a, v, ps, vwv, gv)) continue;  // same outcome and stores in every lane
        const int64_t s = a.xadj[v];
        int pu[R], cu[R];
        group_conn_row<G, R>(a, s, (int)(a.xadj[v + 1] - s), gl, tab, pu, cu);
        uint64_t best = 0;
        int cs = 0, sumB = 0, cntB = 0;
#pragma unroll
        for (int r = 0; r < R; r++) {
            if (cu[r] > 0) {
                if (pu[r] == ps) cs += cu[r];
                else if (a.isB[gv.poff + pu[r]]) {
                    const uint64_t k2 = conn_key(cu[r], pu[r]);
                    best = k2 > best ? k2 : best;
                    sumB += cu[r];
                    cntB++;
                }
            }
        }
        best = gmax_u64<G>(best);
        cs = gsum<G>(cs);
        sumB = gsum<G>(sumB);
        cntB = gsum<G>(cntB);
        if (gl == 0) {
            rb_finish(a, v, ps, gv, best, cs, sumB, cntB, vwv, hmode, lh);
            racc.sel<B>(a, g);
            racc.c0++;
        }
    }
}

template <bool B>
__device__ void rb_blocks(const KArgs &a, int cls, int32_t *tab, int bid, int nblocks, GV &gv, CountX &racc, int hmode,
                          int32_t *lh)
{
    __shared__ uint64_t s_red[BLOCK / 64];
    __shared__ int32_t s_red32[BLOCK / 64];
    const int32_t *list = a.bins + a.binoff[cls];
    const Walk w = walk<B>(a.binoff[cls + 1] - a.binoff[cls], bid, nblocks, 1);
    for (int i = w.first; i < w.end; i += w.step) {
        const int v = list[i];
        const int g = gof<B>(a, v);
        gv.sel<B>(a, g);
        if (!is_rb(gv.kind)) continue;
        const int ps = a.P[v];
        const int vwv = a.vw ? a.vw[v] : 1;
        if (!rb_candidate(a, v, ps, vwv, gv)) continue;
        block_fill(a, v, tab);
        uint64_t best = 0;
        int cs = 0, sumB = 0, cntB = 0;
        for (int p = threadIdx.x; p < gv.k; p += BLOCK) {
            const int c = tab[p];
            if (c) {
                tab[p] = 0;
                if (p == ps) cs = c;
                else if (a.isB[gv.poff + p]) {
                    const uint64_t k2 = conn_key(c, p);
                    best = k2 > best ? k2 : best;
                    sumB += c;
                    cntB++;
                }
            }
        }
        best = block_max_u64<BLOCK>(best, s_red);
        cs = block_sum<BLOCK>(cs, s_red32);
        sumB = block_sum<BLOCK>(sumB, s_red32);
        cntB = block_sum<BLOCK>(cntB, s_red32);
        if (threadIdx.x == 0) {
            rb_finish(a, v, ps, gv, best, cs, sumB, cntB, vwv, hmode, lh);
            racc.sel<B>(a, g);
            racc.c0++;
        }
    }
}

// Small-row role with PC (one graph): the per-part candidate bounds
// 3 (k w(p) - W) (-1 outside A) and the B flags are copied to LDS first, so
// a vertex's candidate test and its neighbours' B tests read LDS instead of
// waiting on dependent global loads.
template <bool B, int ROLE, int GS, int RS, bool PC, int CL, bool PAIR = false>
__device__ __forceinline__ void loss_body(const KArgs &a, int nblk, int hmode)
{
    constexpr bool pcache = PC && !B && ROLE == 1;
    extern __shared__ int32_t lds[];
    const int stride = a.k + 1;
    GV pv, rv;
    CountX racc;
    if (!B) {
        pv.at(a, 0);
        rv.at(a, 0);
        racc.to(a, 0);
    }
    // the block's histogram sits after the role's tables (HIST_LDS, one graph)
    const int hoff = ROLE == 1 ? (BLOCK / GS) * stride + BLOCK : (ROLE == 2 ? (BLOCK / 64) * stride : (ROLE == 3 ? a.k : 0));
    int32_t *lh = lds + hoff;
    if (hmode == HIST_LDS)
        for (int i = threadIdx.x; i < a.k * NSLOT; i += BLOCK) lh[i] = 0;
    if (ROLE == 1) {
        const int ng = BLOCK / GS;
        for (int i = threadIdx.x; i < ng * stride; i += BLOCK) lds[i] = 0;
        const int coff = (hoff + (hmode == HIST_LDS ? a.k * NSLOT : 0) + 1) & ~1;
        int64_t *cthr = reinterpret_cast<int64_t *>(lds + coff);
        uint8_t *cB = reinterpret_cast<uint8_t *>(cthr + a.k);
        if (pcache) {
            const int64_t kk = pv.k;
            for (int p = threadIdx.x; p < a.k; p += BLOCK) {
                cthr[p] = a.isA[p] ? 3 * (kk * a.w[p] - pv.W) : -1;
                cB[p] = a.isB[p];
            }
        }
        __syncthreads();
        int32_t *q = lds + ng * stride + (threadIdx.x >> 6) * 64;
        // one small class per block, as in the gain kernel
        auto body = [&](auto g_c, auto r_c, int cl, int bid, int nb) {
            constexpr int G = decltype(g_c)::value, R = decltype(r_c)::value;
            if (a.tmap[cl] != ROLE) return;
            int32_t *tab = lds + (threadIdx.x / G) * stride;
            const int wid = bid * (BLOCK / 64) + (threadIdx.x >> 6), nwaves = nb * (BLOCK / 64);
            const int32_t *list = (!B && cl == CLS_S && a.sident) ? nullptr : a.bins + a.binoff[cl];
            const Walk wk = walk_q<B>(a, a.binoff[cl + 1] - a.binoff[cl], wid, nwaves, 64, WQ_LOSS + cl);
            auto pre = [&](Meta &m) -> bool {
                    m.g = gof<B>(a, m.v);
                    pv.sel<B>(a, m.g);
                    if (!is_rb(pv.kind)) return false;
                    m.ps = a.P[m.v];
                    m.aux = a.vw ? a.vw[m.v] : 1;
                    if (pcache) {
                        const int64_t x0 = a.xadj[m.v], x1 = a.xadj[m.v + 1];
                        if (2 * (int64_t)pv.k * m.aux > cthr[m.ps]) {
                            rb_no_candidate(a, m.v);
                            return false;
                        }
                        m.s = x0;
                        m.deg = (int)(x1 - x0);
                    } else {
                        if (!rb_candidate(a, m.v, m.ps, m.aux, pv)) return false;
                        m.s = a.xadj[m.v];
                        m.deg = (int)(a.xadj[m.v + 1] - m.s);
                    }
                    if (!PAIR && m.deg <= TINY) {
                        uint64_t best = 0;
                        int sumB = 0, cntB = 0;
                        const int cs = tiny_conn<TINY>(a, m.s, m.deg, m.ps, [&](int p, int c) {
                            if (pcache ? cB[p] : a.isB[pv.poff + p]) {
                                const uint64_t k2 = conn_key(c, p);
                                best = k2 > best ? k2 : best;
                                sumB += c;
                                cntB++;
                            }
                        });
                        rb_finish(a, m.v, m.ps, pv, best, cs, sumB, cntB, m.aux, hmode, lh);
                        racc.sel<B>(a, m.g);
                        racc.c0++;
                        return false;
                    }
                    return true;
                };
            auto row = [&](const Meta &t, int gl) {
                    rv.sel<B>(a, t.g);
                    int pu[R], cu[R];
                    group_conn_row<G, R>(a, t.s, t.deg, gl, tab, pu, cu);
                    uint64_t best = 0;
                    int cs = 0, sumB = 0, cntB = 0;
#pragma unroll
                    for (int r = 0; r < R; r++) {
                        if (cu[r] > 0) {
                            if (pu[r] == t.ps) cs += cu[r];
                            else if (pcache ? cB[pu[r]] : a.isB[rv.poff + pu[r]]) {
                                const uint64_t k2 = conn_key(cu[r], pu[r]);
                                best = k2 > best ? k2 : best;
                                sumB += cu[r];
                                cntB++;
                            }
                        }
                    }
                    best = gmax_u64<G>(best);
                    cs = gsum<G>(cs);
                    sumB = gsum<G>(sumB);
                    cntB = gsum<G>(cntB);
                    if (gl == 0) {
                        rb_finish(a, t.v, t.ps, rv, best, cs, sumB, cntB, t.aux, hmode, lh);
                        racc.sel<B>(a, t.g);
                        racc.c0++;
                    }
                };
            if (PAIR && cl == CLS_S && !a.ew) {
                // two candidate rows per group and round, both rows' parts in flight at once
                auto row2 = [&](const Meta &t0, bool h0, const Meta &t1, bool h1, int gl) {
                    int p0[R], p1[R], cu[R];
                    conn_load<G, R>(a, t0.s, t0.deg, gl, p0);
                    conn_load<G, R>(a, t1.s, t1.deg, gl, p1);
                    auto finish = [&](const Meta &t, const int (&pu)[R]) {
                        rv.sel<B>(a, t.g);
                        conn_claim<R>(tab, pu, cu);
                        uint64_t best = 0;
                        int cs = 0, sumB = 0, cntB = 0;
#pragma unroll
                        for (int r = 0; r < R; r++) {
                            if (cu[r] > 0) {
                                if (pu[r] == t.ps) cs += cu[r];
                                else if (pcache ? cB[pu[r]] : a.isB[rv.poff + pu[r]]) {
                                    const uint64_t k2 = conn_key(cu[r], pu[r]);
                                    best = k2 > best ? k2 : best;
                                    sumB += cu[r];
                                    cntB++;
                                }
                            }
                        }
                        best = gmax_u64<G>(best);
                        cs = gsum<G>(cs);
                        sumB = gsum<G>(sumB);
                        cntB = gsum<G>(cntB);
                        if (gl == 0) {
                            rb_finish(a, t.v, t.ps, rv, best, cs, sumB, cntB, t.aux, hmode, lh);
                            racc.sel<B>(a, t.g);
                            racc.c0++;
                        }
                    };
                    if (h0) finish(t0, p0);
                    if (h1) finish(t1, p1);
                };
                wave_batched2<G>(list, wk, q, pre, row2);
            } else {
                wave_batched<G>(list, wk, q, pre, row);
            }
        };
        if (CL != NCLS) body(std::integral_constant<int, GS>{}, std::integral_constant<int, RS>{}, CL, blockIdx.x, nblk);
        else if ((int)blockIdx.x < a.gS)
            body(std::integral_constant<int, GS>{}, std::integral_constant<int, RS>{}, CLS_S, blockIdx.x, a.gS);
        else
            body(std::integral_constant<int, 8>{}, std::integral_constant<int, 8>{}, CLS_S2, blockIdx.x - a.gS, a.gS2);
    } else if (ROLE == 2) {
        // one wave per candidate row, wave-batched as in the gain kernel
        const int ng = BLOCK / 64;
        for (int i = threadIdx.x; i < ng * stride; i += BLOCK) lds[i] = 0;
        __syncthreads();
        int32_t *tab = lds + (threadIdx.x >> 6) * stride;
        int32_t *q = lds + hoff + (hmode == HIST_LDS ? a.k * NSLOT : 0) + (threadIdx.x >> 6) * 64;
        const int wid = blockIdx.x * ng + (threadIdx.x >> 6), nwaves = nblk * ng;
        const bool scan = a.k <= WAVE_SCAN_KMAX;
        for (int c = 1; c < NCLS; c++) {
            if (a.tmap[c] != 2) continue;
            const int cnt = a.binoff[c + 1] - a.binoff[c];
            const int unit = wave_unit(cnt, nwaves);
            auto pre = [&](Meta &m) -> bool {
                m.g = gof<B>(a, m.v);
                pv.sel<B>(a, m.g);
                if (!is_rb(pv.kind)) return false;
                m.ps = a.P[m.v];
                m.aux = a.vw ? a.vw[m.v] : 1;
                const int64_t x0 = a.xadj[m.v], x1 = a.xadj[m.v + 1];
                if (!rb_candidate(a, m.v, m.ps, m.aux, pv)) return false;
                m.s = x0;
                m.deg = (int)(x1 - x0);
                return true;
            };
            auto row = [&](const Meta &t, int gl) {
                rv.sel<B>(a, t.g);
                uint64_t best = 0;
                int cs = 0, sumB = 0, cntB = 0;
                if (scan) {
                    group_fill_row<64, 16>(a, t.s, t.deg, gl, tab);
                    for (int p = gl; p < rv.k; p += 64) {
                        const int cc = tab[p];
                        if (cc) {
                            tab[p] = 0;
                            if (p == t.ps) cs = cc;
                            else if (a.isB[rv.poff + p]) {
                                const uint64_t k2 = conn_key(cc, p);
                                best = k2 > best ? k2 : best;
                                sumB += cc;
                                cntB++;
                            }
                        }
                    }
                    lds_fence_wave();
                } else {
                    int pu[16], cu[16];
                    group_conn_row<64, 16>(a, t.s, t.deg, gl, tab, pu, cu);
#pragma unroll
                    for (int r = 0; r < 16; r++) {
                        if (cu[r] > 0) {
                            if (pu[r] == t.ps) cs += cu[r];
                            else if (a.isB[rv.poff + pu[r]]) {
                                const uint64_t k2 = conn_key(cu[r], pu[r]);
                                best = k2 > best ? k2 : best;
                                sumB += cu[r];
                                cntB++;
                            }
                        }
                    }
                }
                best = gmax_u64<64>(best);
                cs = gsum<64>(cs);
                sumB = gsum<64>(sumB);
                cntB = gsum<64>(cntB);
                if (gl == 0) {
                    rb_finish(a, t.v, t.ps, rv, best, cs, sumB, cntB, t.aux, hmode, lh);
                    racc.sel<B>(a, t.g);
                    racc.c0++;
                }
            };
            wave_batched<64>(a.bins + a.binoff[c], walk_q<B>(a, cnt, wid, nwaves, unit, WQ_LOSS2 + c), q, pre, row,
                             unit);
        }
    } else if (ROLE == 3) {
        for (int i = threadIdx.x; i < a.k; i += BLOCK) lds[i] = 0;
        __syncthreads();
        for (int c = 1; c < NCLS; c++)
            if (a.tmap[c] == 3) rb_blocks<B>(a, c, lds, blockIdx.x, nblk, pv, racc, hmode, lh);
    } else {
        __syncthreads();
        // isolated vertices: no connectivity, loss 0, random destination (Jetrw)
        const int32_t *list = a.bins + a.binoff[CLS_Z];
        const int cnt = a.binoff[CLS_Z + 1] - a.binoff[CLS_Z];
        int lo, hi;
        block_chunk(cnt, blockIdx.x, nblk, lo, hi);
        for (int i = lo + threadIdx.x; i < hi; i += BLOCK) {
            const int v = list[i];
            const int g = gof<B>(a, v);
            pv.sel<B>(a, g);
            if (!is_rb(pv.kind)) continue;
            const int ps = a.P[v];
            const int vwv = a.vw ? a.vw[v] : 1;
            if (!rb_candidate(a, v, ps, vwv, pv)) continue;
            rb_finish(a, v, ps, pv, 0, 0, 0, 0, vwv, hmode, lh);
            racc.sel<B>(a, g);
            racc.c0++;
        }
    }
    if (hmode == HIST_LDS) {
        __syncthreads();
        for (int i = threadIdx.x; i < a.k * NSLOT; i += BLOCK)
            if (lh[i]) atomicAdd((unsigned long long *)&a.hist[i], (unsigned long long)(int64_t)lh[i]);
    }
    acc_finish(a, racc);
}

template <bool B, int ROLE, int GS = 8, int RS = 32 / GS, bool PC = false, int CL = CLS_S>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(ROLE == 1 && !B ? (CL == CLS_S ? 6 : 8) : 1)))
void k_rb_loss(KArgs a, int nblk, int hmode)
{
    if (!any_rb(a)) return;
    // one graph's small class alone (its own launch): two rows in flight per group
    loss_body<B, ROLE, GS, RS, PC, CL, !B && ROLE == 1 && CL == CLS_S>(a, nblk, hmode);
}

// One launch for the small-row gain and loss passes of one graph: each
// iteration is Jetlp or rebalancing, so a launch runs one of the two and the
// other kind's launch is not needed.
template <int GS, int RS, bool PC, int CL>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(8))) void k_rows(KArgs a, int nblk, int hmode)
{
    if (any_kind(a, KIND_LP)) gain_body<false, 1, GS, RS, CL>(a, nblk);
    else if (any_rb(a)) loss_body<false, 1, GS, RS, PC, CL>(a, nblk, hmode);
}

// Rebalancing loss on long rows, phase 2 (one wave per vertex): the "no
// candidate" outputs, and the candidate rows of more than one chunk.
template <bool B>
__global__ __launch_bounds__(BLOCK) void k_lrb_fin(KArgs a, int hmode)
{
    if (!any_rb(a)) return;
    const int gl = threadIdx.x & 63;
    const int nL = a.binoff[CLS_L + 1] - a.binoff[CLS_L];
    GV pv;
    CountX racc;
    if (!B) {
        pv.at(a, 0);
        racc.to(a, 0);
    }
    const int nw = gridDim.x * (BLOCK / 64);
    for (int li = blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6); li < nL; li += nw) {
        const int v = a.bins[a.binoff[CLS_L] + li];
        const int g = gof<B>(a, v);
        pv.sel<B>(a, g);
        if (!is_rb(pv.kind)) continue;
        const int ps = a.P[v];
        const int vwv = a.vw ? a.vw[v] : 1;
        if (!rb_is_candidate(a, ps, vwv, pv)) {
            if (gl == 0) rb_candidate(a, v, ps, vwv, pv);  // writes the "no candidate" outputs
            continue;
        }
        if (a.xadj[v + 1] - a.xadj[v] <= LCHUNK) continue;  // finished by its chunk's block
        uint64_t best = 0;
        int cs = 0, sumB = 0, cntB = 0;
        for (int p = gl; p < pv.k; p += 64) {
            const int c = chunk_rows_sum(a, li, p);
            if (c) {
                if (p == ps) cs = c;
                else if (a.isB[pv.poff + p]) {
                    const uint64_t k2 = conn_key(c, p);
                    best = k2 > best ? k2 : best;
                    sumB += c;
                    cntB++;
                }
            }
        }
        best = gmax_u64<64>(best);
        cs = gsum<64>(cs);
        sumB = gsum<64>(sumB);
        cntB = gsum<64>(cntB);
        if (gl == 0) {
            rb_finish(a, v, ps, pv, best, cs, sumB, cntB, vwv, hmode, nullptr);
            racc.sel<B>(a, g);
            racc.c0++;
        }
    }
    acc_finish(a, racc);
}

// Per-(part, slot) weight histogram of the candidates. With one graph whose
// k * NSLOT int32 counters fit, each block accumulates its range in LDS and
// adds its nonzero counters once.
template <bool B>
__global__ __launch_bounds__(BLOCK) void k_rb_hist(KArgs a, int use_lds)
{
    extern __shared__ int32_t h[];
    if (!any_rb(a)) return;
    const int nh = a.k * NSLOT;
    if (use_lds) {
        for (int i = threadIdx.x; i < nh; i += BLOCK) h[i] = 0;
        __syncthreads();
    }
    GV pv;
    if (!B) pv.at(a, 0);
    int lo, hi;
    flat_range<B>(a, lo, hi);
    constexpr int U = 4;
    for (int base = lo + threadIdx.x; base < hi; base += BLOCK * U) {
        int vv[U], sl[U], pp[U], ww[U];
#pragma unroll
        for (int j = 0; j < U; j++) {
            const int i = base + j * BLOCK;
            vv[j] = i < hi ? flat_vertex<B>(a, i) : -1;
        }
#pragma unroll
        for (int j = 0; j < U; j++) sl[j] = vv[j] >= 0 ? a.slot[vv[j]] : 255;
#pragma unroll
        for (int j = 0; j < U; j++) {
            pp[j] = sl[j] != 255 ? a.P[vv[j]] : 0;
            ww[j] = sl[j] != 255 ? (a.vw ? a.vw[vv[j]] : 1) : 0;
        }
#pragma unroll
        for (int j = 0; j < U; j++) {
            if (sl[j] == 255) continue;
            pv.sel<B>(a, gof<B>(a, vv[j]));
            if (!is_rb(pv.kind)) continue;  // a slot left from an earlier iteration
            const int idx = (pv.poff + pp[j]) * NSLOT + sl[j];
            if (use_lds) atomicAdd(&h[idx], ww[j]);
            else atomicAdd((unsigned long long *)&a.hist[idx], (unsigned long long)(int64_t)ww[j]);
        }
    }
    if (use_lds) {
        __syncthreads();
        for (int i = threadIdx.x; i < nh; i += BLOCK)
            if (h[i]) atomicAdd((unsigned long long *)&a.hist[i], (unsigned long long)(int64_t)h[i]);
    }
}

// Per graph (one block each): cut-off slot s* of every oversized part (slots
// below it are evicted whole) and the residual weight still needed inside
// s*; Jetrs capacities over B.
__device__ __forceinline__ void part_cutoff(const KArgs &a, int gp, int64_t o, int &ss, int64_t &res)
{
    ss = -1;
    res = 0;
    if (!a.isA[gp]) return;
    const int64_t need = a.w[gp] - o;
    int64_t hv[NSLOT];
#pragma unroll
    for (int s = 0; s < NSLOT; s++) hv[s] = a.hist[(int64_t)gp * NSLOT + s];
    int64_t cum = 0;
    ss = NSLOT;
#pragma unroll
    for (int s = 0; s < NSLOT; s++) {
        if (ss == NSLOT && cum + hv[s] >= need) {
            ss = s;
            res = need - cum;
        }
        cum += hv[s];
    }
}

// Jetrs capacities of graph g: exclusive prefix of sigma - W(b) over its
// list B (whole block).
__device__ void rs_capacities(const KArgs &a, int g, Ctl *c, int64_t *s_scan64)
{
    const int nB = c->nB, poff = c->poff;
    const int64_t sigma = c->sigma;
    int64_t *cap = a.capstart + poff + g;
    int64_t acc = 0;
    for (int base = 0; base < nB; base += BLOCK) {
        const int i = base + threadIdx.x;
        const int64_t cv = i < nB ? sigma - a.w[poff + a.Blist[poff + i]] : 0;
        int64_t tot;
        const int64_t pos = block_excl_scan<BLOCK>(cv, s_scan64, tot);
        if (i < nB) cap[i] = acc + pos;
        acc += tot;
    }
    if (threadIdx.x == 0) {
        cap[nB] = acc;
        c->total_cap = acc;
    }
}

__global__ __launch_bounds__(BLOCK) void k_rb_cutoff(KArgs a)
{
    __shared__ int64_t s_scan64[BLOCK / 64];
    const int g = blockIdx.x;
    Ctl *c = a.ctl + g;
    const int kind = c->kind;
    if (!is_rb(kind)) return;
    const int64_t o = c->o;
    const int k = c->k, poff = c->poff;
    for (int p = threadIdx.x; p < k; p += BLOCK) {
        int ss;
        int64_t res;
        part_cutoff(a, poff + p, o, ss, res);
        a.sstar[poff + p] = ss;
        a.resid[poff + p] = res;
    }
    if (kind == KIND_RS) rs_capacities(a, g, c, s_scan64);
}

// Vertex range [v0, v1) of tile `tile` and its graph's controller.
__device__ __forceinline__ const Ctl *tile_range(const KArgs &a, int tile, int &lt, int &v0, int &v1)
{
    const int g = a.tg ? a.tg[tile] : 0;
    const Ctl *c = a.ctl + g;
    lt = tile - c->t0;
    v0 = c->voff + lt * TILE;
    const int vend = c->voff + c->n;
    v1 = v0 + TILE < vend ? v0 + TILE : vend;
    return c;
}

// Per tile (one block) and part whose cut-off lies inside the histogram:
// weight of the tile's candidates that sit in the part's cut-off slot,
// stored at tsum[rowbase + part * ntiles + tile]. Blocks bid, bid + nb, ...
// take the tiles. With `sst` (one graph, k LDS entries) the blocks first
// find the cut-off slots themselves; block 0 also stores them with the
// residuals and the Jetrs capacities.
__device__ void tilesum_body(const KArgs &a, int bid, int nb, int32_t *acc, int32_t *sst)
{
    __shared__ int64_t s_scan64[BLOCK / 64];
    if (!any_rb(a)) return;
    if (sst) {
        Ctl *c = a.ctl;
        if (!is_rb(c->kind)) return;
        for (int p = threadIdx.x; p < c->k; p += BLOCK) {
            int ss;
            int64_t res;
            part_cutoff(a, p, c->o, ss, res);
            sst[p] = ss;
            if (bid == 0) {
                a.sstar[p] = ss;
                a.resid[p] = res;
            }
        }
        if (bid == 0 && c->kind == KIND_RS) rs_capacities(a, 0, c, s_scan64);
        __syncthreads();
    }
    for (int tile = bid; tile < a.ntile; tile += nb) {
        int lt, v0, v1;
        const Ctl *c = tile_range(a, tile, lt, v0, v1);
        if (!is_rb(c->kind)) continue;
        const int k = c->k, poff = c->poff, ntl = c->ntiles;
        for (int p = threadIdx.x; p < k; p += BLOCK) acc[p] = 0;
        __syncthreads();
        {
            int sl[PER], pp[PER], ss[PER];
#pragma unroll
            for (int j = 0; j < PER; j++) {
                const int v = v0 + threadIdx.x + j * BLOCK;
                sl[j] = v < v1 ? a.slot[v] : 255;
            }
#pragma unroll
            for (int j = 0; j < PER; j++) pp[j] = sl[j] != 255 ? a.P[v0 + threadIdx.x + j * BLOCK] : 0;
#pragma unroll
            for (int j = 0; j < PER; j++) ss[j] = sl[j] != 255 ? (sst ? sst[pp[j]] : a.sstar[poff + pp[j]]) : -1;
#pragma unroll
            for (int j = 0; j < PER; j++)
                if (sl[j] != 255 && sl[j] == ss[j])
                    atomicAdd(&acc[pp[j]], a.vw ? a.vw[v0 + threadIdx.x + j * BLOCK] : 1);
        }
        __syncthreads();
        int32_t *row = a.tsum + c->rowbase + lt;
        for (int p = threadIdx.x; p < k; p += BLOCK) {
            const int ss = sst ? sst[p] : a.sstar[poff + p];
            if (ss >= 0 && ss < NSLOT) row[(int64_t)p * ntl] = acc[p];
        }
        __syncthreads();
    }
}

// One launch for two passes that never run in the same iteration of a
// graph: blocks [0, nafter) run the afterburner (Jetlp), the rest the tile
// sums of the rebalancing selection. Dynamic LDS: k ints, 2k when the
// cut-off is found here (fuse_cut, one graph).
template <bool B>
__global__ __launch_bounds__(BLOCK) void k_after_tsum(KArgs a, int nafter, int fuse_cut)
{
    extern __shared__ int32_t lds[];
    if ((int)blockIdx.x < nafter) afterburner_body<B>(a, blockIdx.x);
    else tilesum_body(a, blockIdx.x - nafter, gridDim.x - nafter, lds, fuse_cut ? lds + a.k : nullptr);
}

// Per part whose cut-off lies inside the histogram (one block): an exclusive
// scan of its tile sums finds the one tile in which the running cut-off-slot
// weight reaches the residual (every cut-off-slot vertex of an earlier tile
// is evicted, none of a later one). Inside that tile the vertices are taken
// in id order while the weight before them is below the residual; the last
// evicted id is the part's threshold.
__global__ __launch_bounds__(BLOCK) void k_rb_split(KArgs a)
{
    __shared__ int64_t s_scan[BLOCK / 64];
    __shared__ uint64_t s_red[BLOCK / 64];
    __shared__ int s_tile;
    __shared__ int64_t s_base;
    if (!any_rb(a)) return;
    for (int gp = blockIdx.x; gp < a.ktot; gp += gridDim.x) {
        const int g = a.pg ? a.pg[gp] : 0;
        const Ctl *c = a.ctl + g;
        if (!is_rb(c->kind)) continue;
        const int ss = a.sstar[gp];
        if (ss < 0 || ss >= NSLOT) continue;
        const int p = gp - c->poff, ntl = c->ntiles;
        const int32_t *row = a.tsum + c->rowbase + (int64_t)p * ntl;
        const int64_t resid = a.resid[gp];
        if (threadIdx.x == 0) s_tile = -1;
        __syncthreads();
        int64_t carry = 0;
        for (int b0 = 0; b0 < ntl; b0 += BLOCK) {
            const int i = b0 + threadIdx.x;
            const int64_t x = i < ntl ? row[i] : 0;
            int64_t tot;
            const int64_t before = carry + block_excl_scan<BLOCK>(x, s_scan, tot);
            if (x > 0 && before < resid && resid <= before + x) {
                s_tile = i;
                s_base = before;
            }
            carry += tot;
        }
        __syncthreads();
        const int lt = s_tile;
        uint64_t last = 0;  // (last evicted id + 1), 0 = none
        if (lt >= 0) {
            const int vbeg = c->voff + lt * TILE, vend0 = c->voff + c->n;
            const int vend = vbeg + TILE < vend0 ? vbeg + TILE : vend0;
            const int v0 = vbeg + threadIdx.x * PER;
            int wv[PER];
            int64_t mine = 0;
#pragma unroll
            for (int q = 0; q < PER; q++) {
                const int v = v0 + q;
                wv[q] = 0;
                if (v < vend && a.slot[v] == ss && a.P[v] == p) wv[q] = a.vw ? a.vw[v] : 1;
                mine += wv[q];
            }
            int64_t tot;
            int64_t before = s_base + block_excl_scan<BLOCK>(mine, s_scan, tot);
#pragma unroll
            for (int q = 0; q < PER; q++) {
                if (wv[q] > 0 && before < resid) last = (uint64_t)(v0 + q) + 1;
                before += wv[q];
            }
        }
        last = block_max_u64<BLOCK>(last, s_red);
        if (threadIdx.x == 0) a.vthr[gp] = (int32_t)last - 1;
        __syncthreads();
    }
}

// Eviction decision for every candidate (one block per tile): evicted when
// its slot is below the part's cut-off, or equal with an id no larger than
// the part's threshold. Jetrw moves it to its chosen destination; Jetrs marks
// it and sums the tile's evicted weight.
__global__ __launch_bounds__(BLOCK) void k_rb_mark(KArgs a)
{
    __shared__ int64_t s_red[BLOCK / 64];
    if (!any_rb(a)) return;
    for (int tile = blockIdx.x; tile < a.ntile; tile += gridDim.x) {
        int lt, v0, v1;
        const Ctl *c = tile_range(a, tile, lt, v0, v1);
        const int kind = c->kind;
        if (!is_rb(kind)) continue;
        const int poff = c->poff;
        int64_t es = 0;
        int sl[PER], gp[PER], ss[PER], th[PER];
#pragma unroll
        for (int j = 0; j < PER; j++) {
            const int v = v0 + threadIdx.x + j * BLOCK;
            sl[j] = v < v1 ? a.slot[v] : 255;
        }
#pragma unroll
        for (int j = 0; j < PER; j++) gp[j] = sl[j] != 255 ? poff + a.P[v0 + threadIdx.x + j * BLOCK] : -1;
#pragma unroll
        for (int j = 0; j < PER; j++) {
            ss[j] = gp[j] >= 0 ? a.sstar[gp[j]] : -1;
            th[j] = gp[j] >= 0 ? a.vthr[gp[j]] : -1;
        }
#pragma unroll
        for (int j = 0; j < PER; j++) {
            const int v = v0 + threadIdx.x + j * BLOCK;
            if (v >= v1) continue;
            const bool ev = sl[j] != 255 && (sl[j] < ss[j] || (sl[j] == ss[j] && v <= th[j]));
            if (kind == KIND_RW) {
                if (ev) {
                    const int d = a.rbd[v];
                    a.dest[v] = d;
                    mq_set(a, v, gp[j] - poff, d);
                }
            } else {
                a.rsev[v] = ev;
                if (ev) es += a.vw ? a.vw[v] : 1;
            }
        }
        if (kind == KIND_RS) {
            es = block_sum<BLOCK>(es, s_red);
            if (threadIdx.x == 0) a.esum[tile] = es;
        }
    }
}

// Jetrs cookie-cutter (one block per tile, PER consecutive vertices per
// thread): evicted vertices in id order take consecutive positions (exclusive
// prefix of their weights); position pos goes to the valid destination whose
// capacity interval [capstart, capstart + cap) holds it; positions beyond the
// total capacity stay.
__global__ __launch_bounds__(BLOCK) void k_rs_assign(KArgs a)
{
    __shared__ int64_t s_scan[BLOCK / 64];
    __shared__ int64_t s_red[BLOCK / 64];
    if (!any_kind(a, KIND_RS)) return;
    for (int tile = blockIdx.x; tile < a.ntile; tile += gridDim.x) {
        int lt, v0, v1;
        const Ctl *c = tile_range(a, tile, lt, v0, v1);
        if (c->kind != KIND_RS) continue;
        const int g = a.tg ? a.tg[tile] : 0;
        const int nB = c->nB, poff = c->poff;
        const int64_t total = c->total_cap;
        const int64_t *cap = a.capstart + poff + g;
        const int vb = v0 + threadIdx.x * PER;
        int wv[PER];
        int64_t mine = 0;
#pragma unroll
        for (int q = 0; q < PER; q++) {
            const int v = vb + q;
            wv[q] = (v < v1 && a.rsev[v]) ? (a.vw ? a.vw[v] : 1) : 0;
            mine += wv[q];
        }
        // evicted weight of the graph's earlier tiles
        int64_t before = 0;
        for (int t = c->t0 + threadIdx.x; t < tile; t += BLOCK) before += a.esum[t];
        before = block_sum<BLOCK>(before, s_red);
        int64_t tot;
        int64_t pos = before + block_excl_scan<BLOCK>(mine, s_scan, tot);
#pragma unroll
        for (int q = 0; q < PER; q++) {
            if (wv[q] > 0 && pos < total) {
                int lo = 0, hi = nB;  // largest i with cap[i] <= pos (cap[0] = 0 <= pos)
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (cap[mid] <= pos) lo = mid;
                    else hi = mid;
                }
                const int d = a.Blist[poff + lo];
                a.dest[vb + q] = d;
                mq_set(a, vb + q, a.P[vb + q], d);
            }
            pos += wv[q];
        }
    }
}

// ------------------------------------------- persistent connectivity table --
// Section 4.3's vertex-part connectivity structure, kept across iterations
// (JET_F_CONN_TABLE, one graph). Row v owns min(k, deg v) slots (the
// paper's space bound); its first tsize[v] slots form an open-addressed hash
// table keyed by part (linear probing), sized a little above the number of
// parts v touched when the row was last built. A slot holds
// (count << 32) | part, or TAB_EMPTY. A part whose count falls to zero keeps
// its slot until the row is rebuilt.
//  * Build (set-up; after an iteration that moved more than a tenth of the
//    vertices; for flagged rows otherwise): the row's part counts in LDS,
//    then its nonzero parts inserted by CAS into the cleared row.
//  * Update (Algorithm 6), after the cut delta of an iteration that moved at
//    most a tenth: every moved vertex's edge weights leave its source part
//    and join its destination part in its neighbours' rows, inserting the
//    part where missing; a row with no free slot for an insert is listed and
//    rebuilt after the moves, with more slots (the paper's failed-insert
//    rehash).
//  * Gains and losses scan rows instead of gathering neighbour parts. The
//    maximum is taken on (count, ~part) keys, so slot order (and the races
//    that decide it) never changes a result.
constexpr unsigned long long TAB_EMPTY = 0xFFFFFFFFull;

__device__ __forceinline__ int tab_part(unsigned long long x) { return (int)(uint32_t)x; }  // -1: empty
__device__ __forceinline__ int tab_cnt(unsigned long long x) { return (int)(x >> 32); }
__device__ __forceinline__ int tab_home(int p, int size) { return (int)(((uint32_t)p * 2654435761u) % (uint32_t)size); }

// Slots a row is built with for nz nonzero parts (at most its allocation).
__device__ __forceinline__ int tab_size(int nz, int alloc)
{
    const int want = nz + (nz / 4 > 2 ? nz / 4 : 2);
    return want < alloc ? want : alloc;
}

// Adds w to part p of a row of `size` slots, inserting p in a free slot if
// absent; false when no slot is free.
__device__ __forceinline__ bool tab_add(unsigned long long *row, int size, int p, int w)
{
    const unsigned long long inc = (unsigned long long)(uint32_t)w << 32;
    int i = tab_home(p, size);
    for (int n = 0; n < size; n++) {
        const unsigned long long x = row[i];
        if (tab_part(x) == p) {
            atomicAdd(&row[i], inc);
            return true;
        }
        if (x == TAB_EMPTY) {
            const unsigned long long old = atomicCAS(&row[i], TAB_EMPTY, inc | (uint32_t)p);
            if (old == TAB_EMPTY) return true;
            if (tab_part(old) == p) {
                atomicAdd(&row[i], inc);
                return true;
            }
        }
        i = i + 1 == size ? 0 : i + 1;
    }
    return false;
}

// Subtracts w from part p of a row (p is present: a moved neighbour was in p).
__device__ __forceinline__ void tab_sub(unsigned long long *row, int size, int p, int w)
{
    const unsigned long long dec = (unsigned long long)(-(int64_t)((uint64_t)(uint32_t)w << 32));
    int i = tab_home(p, size);
    for (int n = 0; n < size; n++) {
        if (tab_part(row[i]) == p) {
            atomicAdd(&row[i], dec);
            return;
        }
        i = i + 1 == size ? 0 : i + 1;
    }
}

// Writes the counts a group of G lanes holds (pu / cu as from
// group_conn_row: each nonzero part once, with its connectivity) into row v:
// sizes the row, clears it, inserts.
template <int G, int R>
__device__ __forceinline__ void tab_store_row(const KArgs &a, int v, int gl, const int (&pu)[R], const int (&cu)[R])
{
    int nz = 0;
#pragma unroll
    for (int r = 0; r < R; r++) nz += cu[r] > 0;
    nz = gsum<G>(nz);
    const int64_t s = a.toff[v];
    const int alloc = (int)(a.toff[v + 1] - s);
    const int size = tab_size(nz, alloc);
    unsigned long long *row = a.tab + s;
    for (int i = gl; i < size; i += G) row[i] = TAB_EMPTY;
    if (gl == 0) a.tsize[v] = size;
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < R; r++)
        if (cu[r] > 0) tab_add(row, size, pu[r], cu[r]);
}

// Role of a class in the table build: that of the gain pass (a.tmap: 1
// groups of 8 lanes, 2 one wave, 3 one block per row, chosen by k so the
// LDS tables fit), long rows always one block.
__device__ __forceinline__ int tab_role(const KArgs &a, int cls) { return cls == CLS_L || a.tmap[cls] == 0 ? 3 : a.tmap[cls]; }

// Builds rows: every row (at set-up, or after an iteration that moved more
// than a tenth of the vertices) or the listed ones (after smaller move
// sets); nothing after an iteration without moves. One graph.
template <int ROLE>
__global__ __launch_bounds__(BLOCK) void k_tab_build(KArgs a, int setup)
{
    extern __shared__ int32_t lds[];
    __shared__ int32_t s_red32[BLOCK / 64];
    bool full = setup != 0;
    if (!full) {
        if (!any_active(a)) return;
        int64_t moved = 0;
        for (int i = 0; i < NSHARD; i++) moved += a.bstat[ST_M * NSHARD + i];
        if (moved == 0) return;
        full = 10 * moved > (int64_t)a.n;
        if (!full && a.cnt[CNT_TFAIL] == 0) return;
    }
    constexpr int G = ROLE == 1 ? 8 : 64, R = ROLE == 1 ? 8 : 16;
    const int stride = a.k + 1;
    const int ntab = ROLE == 1 ? BLOCK / 8 : (ROLE == 2 ? BLOCK / 64 : 1);
    for (int i = threadIdx.x; i < ntab * (ROLE == 3 ? a.k : stride); i += BLOCK) lds[i] = 0;
    __syncthreads();
    // one row: counts in LDS, then the row written
    auto group_row = [&](int v, int gl, int32_t *tab) {
        const int64_t s = a.xadj[v];
        int pu[R], cu[R];
        group_conn_row<G, R>(a, s, (int)(a.xadj[v + 1] - s), gl, tab, pu, cu);
        tab_store_row<G, R>(a, v, gl, pu, cu);
        if (gl == 0) a.tfail[v] = 0;
    };
    auto block_row = [&](int v) {
        block_fill(a, v, lds);
        int nz = 0;
        for (int p = threadIdx.x; p < a.k; p += BLOCK) nz += lds[p] > 0;
        nz = block_sum<BLOCK>(nz, s_red32);
        const int64_t s = a.toff[v];
        const int size = tab_size(nz, (int)(a.toff[v + 1] - s));
        unsigned long long *row = a.tab + s;
        for (int j = threadIdx.x; j < size; j += BLOCK) row[j] = TAB_EMPTY;
        if (threadIdx.x == 0) {
            a.tsize[v] = size;
            a.tfail[v] = 0;
        }
        __syncthreads();
        for (int p = threadIdx.x; p < a.k; p += BLOCK) {
            const int c = lds[p];
            if (c) {
                lds[p] = 0;
                tab_add(row, size, p, c);
            }
        }
        __syncthreads();
    };
    if (ROLE == 3) {
        if (full) {
            for (int c = CLS_S; c <= CLS_L; c++) {
                if (tab_role(a, c) != 3) continue;
                const int32_t *list = a.bins + a.binoff[c];
                const int cnt = a.binoff[c + 1] - a.binoff[c];
                for (int i = blockIdx.x; i < cnt; i += gridDim.x) block_row(list[i]);
            }
        } else {
            const int cnt = a.cnt[CNT_TFAIL];
            for (int i = blockIdx.x; i < cnt; i += gridDim.x) {
                const int v = a.tlist[i];
                if (tab_role(a, degree_class(a.xadj[v + 1] - a.xadj[v])) == 3) block_row(v);
            }
        }
        return;
    }
    int32_t *tab = lds + (threadIdx.x / G) * stride;
    const int gl = threadIdx.x & (G - 1);
    const int gid = blockIdx.x * (BLOCK / G) + threadIdx.x / G, ngr = gridDim.x * (BLOCK / G);
    if (full) {
        for (int c = CLS_S; c <= CLS_M; c++) {
            if (tab_role(a, c) != ROLE) continue;
            const int32_t *list = a.bins + a.binoff[c];
            const int cnt = a.binoff[c + 1] - a.binoff[c];
            for (int i = gid; i < cnt; i += ngr) group_row(list[i], gl, tab);
        }
    } else {
        const int cnt = a.cnt[CNT_TFAIL];
        for (int i = gid; i < cnt; i += ngr) {
            const int v = a.tlist[i];
            if (tab_role(a, degree_class(a.xadj[v + 1] - a.xadj[v])) == ROLE) group_row(v, gl, tab);
        }
    }
}

// Jetlp gain (RB = false) or rebalancing loss (RB = true) from the rows:
// rows of up to 64 slots in groups of 8 lanes, longer rows one wave each;
// lanes first inspect 64 list entries at once (wave-batched).
template <bool RB, int G>
__device__ __forceinline__ void tab_scan_class(const KArgs &a, int cls, int wid, int nwaves, int32_t *q, GV &pv,
                                               GainPre &pacc, CountX &racc, int hmode)
{
    const int cnt = a.binoff[cls + 1] - a.binoff[cls];
    const int unit = G == 64 ? wave_unit(cnt, nwaves) : 64;
    auto pre = [&](Meta &m) -> bool {
        if (RB) {
            if (!is_rb(pv.kind)) return false;
            m.ps = a.P[m.v];
            m.aux = a.vw ? a.vw[m.v] : 1;
            const int64_t t0 = a.toff[m.v];
            const int sz = a.tsize[m.v];
            if (!rb_candidate(a, m.v, m.ps, m.aux, pv)) return false;
            m.s = t0;
            m.deg = sz;
            return true;
        }
        if (pv.kind != KIND_LP) return false;
        m.ps = a.P[m.v];
        const int lk = a.lock[m.v];
        const int64_t t0 = a.toff[m.v];
        const int sz = a.tsize[m.v];
        pacc.c0++;
        if (lk == pv.lp_id - 1) {
            gain_locked(a, m.v, m.ps);
            return false;
        }
        m.s = t0;
        m.deg = sz;
        pacc.c1++;
        pacc.c2 += sz;
        return true;
    };
    auto row = [&](const Meta &t, int gl) {
        uint64_t best = 0;
        int cs = 0, sumB = 0, cntB = 0;
        for (int i = gl; i < t.deg; i += G) {
            const unsigned long long x = a.tab[t.s + i];
            const int c = tab_cnt(x), p = tab_part(x);
            if (x == TAB_EMPTY || c == 0) continue;
            if (p == t.ps) cs = c;
            else if (!RB || a.isB[p]) {
                const uint64_t k2 = conn_key(c, p);
                best = k2 > best ? k2 : best;
                sumB += c;
                cntB++;
            }
        }
        best = gmax_u64<G>(best);
        cs = gsum<G>(cs);
        if (RB) {
            sumB = gsum<G>(sumB);
            cntB = gsum<G>(cntB);
        }
        if (gl == 0) {
            if (RB) {
                rb_finish(a, t.v, t.ps, pv, best, cs, sumB, cntB, t.aux, hmode, nullptr);
                racc.c0++;
            } else {
                racc.c0 += gain_finish(a, t.v, t.ps, best, cs, pv.cn, pv.cd);
            }
        }
    };
    wave_batched<G>(a.bins + a.binoff[cls], walk<false>(cnt, wid, nwaves, unit), q, pre, row, unit);
}

template <bool RB>
__global__ __launch_bounds__(BLOCK) void k_tab_scan(KArgs a, int gS)
{
    __shared__ int32_t s_q[BLOCK];
    if (RB ? !any_rb(a) : !any_kind(a, KIND_LP)) return;
    GV pv;
    GainPre pacc;
    CountX racc;
    pv.at(a, 0);
    pacc.to(a, 0);
    racc.to(a, 0);
    int32_t *q = s_q + (threadIdx.x >> 6) * 64;
    // blocks [0, gS): the small classes (groups of 8 lanes); the rest: medium and long rows
    if ((int)blockIdx.x < gS) {
        const int wid = blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6), nw = gS * (BLOCK / 64);
        tab_scan_class<RB, 8>(a, CLS_S, wid, nw, q, pv, pacc, racc, HIST_NONE);
        tab_scan_class<RB, 8>(a, CLS_S2, wid, nw, q, pv, pacc, racc, HIST_NONE);
        if (RB && is_rb(pv.kind)) {
            // isolated candidates: no connectivity, loss 0, random destination (Jetrw)
            const int32_t *list = a.bins + a.binoff[CLS_Z];
            const int cnt = a.binoff[CLS_Z + 1] - a.binoff[CLS_Z];
            for (int i = blockIdx.x * BLOCK + threadIdx.x; i < cnt; i += gS * BLOCK) {
                const int v = list[i];
                const int ps = a.P[v];
                const int vwv = a.vw ? a.vw[v] : 1;
                if (!rb_candidate(a, v, ps, vwv, pv)) continue;
                rb_finish(a, v, ps, pv, 0, 0, 0, 0, vwv, HIST_NONE, nullptr);
                racc.c0++;
            }
        }
    } else {
        const int nb = gridDim.x - gS;
        const int wid = (blockIdx.x - gS) * (BLOCK / 64) + (threadIdx.x >> 6), nw = nb * (BLOCK / 64);
        tab_scan_class<RB, 64>(a, CLS_M, wid, nw, q, pv, pacc, racc, HIST_NONE);
        tab_scan_class<RB, 64>(a, CLS_L, wid, nw, q, pv, pacc, racc, HIST_NONE);
    }
    if (!RB) acc_finish(a, pacc);
    acc_finish(a, racc);
}

// Algorithm 6 on one moved row: every neighbour's row loses w in the source
// part and gains it in the destination part. The paper runs the two halves
// as separate passes so that the first can open slots the second reuses;
// here a slot whose count reached zero keeps its part until the row is
// rebuilt, so the decrements and increments of all moves commute (a count
// never goes below zero: the source part held at least w) and one pass
// does both.
__device__ __forceinline__ void tab_update_row(const KArgs &a, int64_t s, int deg, int ps, int pn, int gl, int stride)
{
    for (int i = gl; i < deg; i += stride) {
        const int u = ld_adj(a, s + i);
        const int w = ld_ew(a, s + i);
        unsigned long long *row = a.tab + a.toff[u];
        const int size = a.tsize[u];
        tab_sub(row, size, ps, w);
        if (!tab_add(row, size, pn, w)) {
            // no slot left: the row is rebuilt after the moves
            if (atomicExch(&a.tfail[u], 1) == 0) a.tlist[atomicAdd(&a.cnt[CNT_TFAIL], 1)] = u;
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_tab_update(KArgs a, int gS)
{
    __shared__ int32_t s_q[BLOCK];
    if (!any_active(a)) return;
    // more than a tenth of the vertices moved: the whole table is rebuilt instead
    int64_t moved = 0;
    for (int i = 0; i < NSHARD; i++) moved += a.bstat[ST_M * NSHARD + i];
    if (moved == 0 || 10 * moved > (int64_t)a.n) return;
    int32_t *q = s_q + (threadIdx.x >> 6) * 64;
    auto pre = [&](Meta &m) -> bool {
        const int pn = a.dest[m.v];
        if (pn < 0) return false;
        m.aux = pn;
        m.ps = a.P[m.v];
        m.s = a.xadj[m.v];
        m.deg = (int)(a.xadj[m.v + 1] - m.s);
        return true;
    };
    if ((int)blockIdx.x < gS) {
        const int wid = blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6), nw = gS * (BLOCK / 64);
        wave_batched<8>(a.bins + a.binoff[CLS_S], walk<false>(a.binoff[CLS_S2 + 1] - a.binoff[CLS_S], wid, nw, 64), q,
                        pre, [&](const Meta &t, int gl) { tab_update_row(a, t.s, t.deg, t.ps, t.aux, gl, 8); });
    } else {
        const int nb = gridDim.x - gS;
        const int wid = (blockIdx.x - gS) * (BLOCK / 64) + (threadIdx.x >> 6), nw = nb * (BLOCK / 64);
        const int cnt = a.binoff[CLS_L + 1] - a.binoff[CLS_M];
        const int unit = wave_unit(cnt, nw);
        wave_batched<64>(a.bins + a.binoff[CLS_M], walk<false>(cnt, wid, nw, unit), q, pre,
                         [&](const Meta &t, int gl) { tab_update_row(a, t.s, t.deg, t.ps, t.aux, gl, 64); },
                         unit);
    }
}

// Row offsets of the table: prefix sums of min(k, deg v), in three passes
// (block sums, their scan, the fill). Blocks own contiguous vertex ranges.
__global__ __launch_bounds__(BLOCK) void k_toff_count(const int64_t *xadj, int n, int k, int64_t *blk)
{
    __shared__ int64_t s_red[BLOCK / 64];
    int lo, hi;
    block_chunk(n, blockIdx.x, gridDim.x, lo, hi);
    int64_t sum = 0;
    for (int v = lo + threadIdx.x; v < hi; v += BLOCK) {
        const int64_t d = xadj[v + 1] - xadj[v];
        sum += d < k ? d : k;
    }
    sum = block_sum<BLOCK>(sum, s_red);
    if (threadIdx.x == 0) blk[blockIdx.x] = sum;
}

__global__ __launch_bounds__(BLOCK) void k_toff_scan(int64_t *blk, int nblk)
{
    __shared__ int64_t s_scan[BLOCK / 64];
    int64_t carry = 0;
    for (int b0 = 0; b0 < nblk; b0 += BLOCK) {
        const int i = b0 + threadIdx.x;
        const int64_t x = i < nblk ? blk[i] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan<BLOCK>(x, s_scan, tot);
        if (i < nblk) blk[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) blk[nblk] = carry;
}

__global__ __launch_bounds__(BLOCK) void k_toff_fill(const int64_t *xadj, int n, int k, const int64_t *blk, int64_t *toff)
{
    __shared__ int64_t s_scan[BLOCK / 64];
    int lo, hi;
    block_chunk(n, blockIdx.x, gridDim.x, lo, hi);
    int64_t carry = blk[blockIdx.x];
    for (int b0 = lo; b0 < hi; b0 += BLOCK) {
        const int v = b0 + threadIdx.x;
        int64_t x = 0;
        if (v < hi) {
            const int64_t d = xadj[v + 1] - xadj[v];
            x = d < k ? d : k;
        }
        int64_t tot;
        const int64_t ex = block_excl_scan<BLOCK>(x, s_scan, tot);
        if (v < hi) toff[v] = carry + ex;
        carry += tot;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) toff[n] = blk[gridDim.x];
}

// ------------------------------------------------------ gather ceiling ----
// The floor of any pass that reads every CSR entry (neighbour id, edge
// weight) and gathers its neighbour's part: one pass with nothing else, 16
// entries per thread (all loads before the gathers, the entries streamed
// with non-temporal loads as the row passes stream them), the partition as
// refinement holds it (T = uint8_t for k <= 256, else uint16_t). Timed by
// jet_gather_ceiling.
template <class T>
__global__ __launch_bounds__(BLOCK) void k_gather_ceiling(const int32_t *adj, const int32_t *ew, const T *P,
                                                          int64_t nnz, unsigned long long *out)
{
    constexpr int U = 16;
    uint32_t acc = 0;
    const int64_t stride = (int64_t)gridDim.x * BLOCK * U;
    for (int64_t base = (int64_t)blockIdx.x * BLOCK * U + threadIdx.x; base < nnz; base += stride) {
        int u[U], w[U];
#pragma unroll
        for (int j = 0; j < U; j++) {
            const int64_t i = base + (int64_t)j * BLOCK;
            u[j] = i < nnz ? __builtin_nontemporal_load(adj + i) : -1;
            w[j] = i < nnz ? (ew ? __builtin_nontemporal_load(ew + i) : 1) : 0;
        }
#pragma unroll
        for (int j = 0; j < U; j++) acc += u[j] >= 0 ? (uint32_t)P[u[j]] * (uint32_t)w[j] : 0u;
    }
    acc = gsum<64>(acc);
    if ((threadIdx.x & 63) == 0 && acc) atomicAdd(out, (unsigned long long)acc);
}

template <class T>
__global__ __launch_bounds__(BLOCK) void k_part_narrow(const int32_t *part, int n, T *P)
{
    for (int v = blockIdx.x * BLOCK + threadIdx.x; v < n; v += gridDim.x * BLOCK) P[v] = (T)part[v];
}

// --------------------------------------------------------- batch autotuner --
// A dry-run copy of the batch's state for timing the gain pass: every graph
// in a Jetlp iteration with nothing locked (its lock stamps are all -1 at
// set-up), a count row saying so. The tuner's passes write their records and
// counters into scratch; the real state is untouched.
__global__ __launch_bounds__(BLOCK) void k_tune_prep(KArgs a, Ctl *ctl2, int32_t *cnt2)
{
    const int g = blockIdx.x;
    if (threadIdx.x == 0) {
        Ctl c = a.ctl[g];
        c.kind = KIND_LP;
        if (c.lp_id < 1) c.lp_id = 1;
        ctl2[g] = c;
    }
    if (g == 0)
        for (int i = threadIdx.x; i < CNT_N + 2; i += BLOCK) cnt2[i] = i == CNT_ROW + KIND_LP ? a.ngraph : 0;
}

// ------------------------------------------------------- batch union graph --

// One graph of a batch as the union sees it.
struct UDesc {
    const int64_t *xadj;
    const int32_t *adj, *vw, *ew;
    int32_t *part;
    int64_t eoff, nnz;
    int32_t voff, n, ret_iter, pad;
};

// Graph whose range [off(g), off(g + 1)) holds x (binary search over G).
template <class Off>
__device__ __forceinline__ int find_graph(int G, int64_t x, Off off)
{
    int lo = 0, hi = G;  // off(lo) <= x < off(hi)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off(mid) <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Union vertex arrays: row offsets shifted by the graph's first CSR entry,
// vertex weights, graph ids and P_0 (also the start of P_best). Checks each
// graph's first and last row offset. Blocks own contiguous ranges.
__global__ __launch_bounds__(BLOCK) void k_union_vertices(const UDesc *d, int G, int N, int64_t NNZ, int64_t *xadj,
                                                          int32_t *vw, int32_t *vg, int32_t *p0, int32_t *bad)
{
    int lo, hi;
    block_chunk(N, blockIdx.x, gridDim.x, lo, hi);
    if (lo >= hi) return;
    int g = find_graph(G, lo + threadIdx.x, [&](int i) { return (int64_t)d[i].voff; });
    for (int v = lo + threadIdx.x; v < hi; v += BLOCK) {
        while (g + 1 < G && v >= d[g + 1].voff) g++;
        const UDesc &u = d[g];
        const int i = v - u.voff;
        const int64_t x = u.xadj[i];
        xadj[v] = x + u.eoff;
        if (vw) vw[v] = u.vw ? u.vw[i] : 1;
        vg[v] = g;
        p0[v] = u.part[i];
        if (i == 0 && (x != 0 || u.xadj[u.n] != u.nnz)) *bad = 1;
        if (v == N - 1) xadj[N] = NNZ;
    }
}

// Union edge arrays: neighbour ids shifted by the graph's first vertex (each
// checked against the graph's own range) and edge weights.
__global__ __launch_bounds__(BLOCK) void k_union_edges(const UDesc *d, int G, int64_t NNZ, int32_t *adj, int32_t *ew,
                                                       int32_t *bad)
{
    const int64_t per = ((NNZ + gridDim.x - 1) / gridDim.x + BLOCK - 1) / BLOCK * BLOCK;
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = lo + per < NNZ ? lo + per : NNZ;
    if (lo >= hi) return;
    int g = find_graph(G, lo + threadIdx.x, [&](int i) { return d[i].eoff; });
    int badl = 0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += BLOCK) {
        while (g + 1 < G && e >= d[g + 1].eoff) g++;
        const UDesc &u = d[g];
        const int64_t i = e - u.eoff;
        const int x = u.adj[i];
        if (x < 0 || x >= u.n) badl = 1;
        adj[e] = x + u.voff;
        if (ew) ew[e] = u.ew ? u.ew[i] : 1;
    }
    if (badl) *bad = 1;
}

// Result of each graph back into the caller's array: P_best, or P_iter for
// graphs that asked for it.
__global__ __launch_bounds__(BLOCK) void k_union_scatter(const UDesc *d, int G, int N, const uint16_t *P,
                                                         const int32_t *best)
{
    int lo, hi;
    block_chunk(N, blockIdx.x, gridDim.x, lo, hi);
    if (lo >= hi) return;
    int g = find_graph(G, lo + threadIdx.x, [&](int i) { return (int64_t)d[i].voff; });
    for (int v = lo + threadIdx.x; v < hi; v += BLOCK) {
        while (g + 1 < G && v >= d[g + 1].voff) g++;
        const UDesc &u = d[g];
        u.part[v - u.voff] = u.ret_iter ? P[v] : best[v];
    }
}

// ------------------------------------------------------------- host side --

int hip_status(jet_context *ctx, hipError_t e)
{
    if (e == hipSuccess) return JET_OK;
    ctx->last_hip = (int)e;
    if (e == hipErrorOutOfMemory) return JET_ENOMEM;
    return JET_EHIP;
}

void *ws_get(jet_context *ctx, int slot, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    if (ctx->scratch_on) {
        // jet_refine_noalloc: bump allocation from the static scratch array;
        // every slot is requested once per call
        const size_t off = (ctx->scratch_off + 255) & ~(size_t)255;
        if (!ctx->scratch || off + bytes > (size_t)JET_NOALLOC_SCRATCH_BYTES) return nullptr;
        ctx->scratch_off = off + bytes;
        return ctx->scratch + off;
    }
    Buffer &b = ctx->bufs[slot];
    if (b.bytes >= bytes) return b.ptr;
    if (b.ptr) {
        (void)hipFree(b.ptr);
        b.ptr = nullptr;
        b.bytes = 0;
    }
    // geometric growth: a context serving graphs of rising sizes reallocates
    // a slot only a few times (every hipFree waits for the whole device)
    size_t want = std::max(bytes + bytes / 8, b.bytes * 2);
    if (hipMalloc(&b.ptr, want) != hipSuccess) {
        (void)hipGetLastError();
        b.ptr = nullptr;
        return nullptr;
    }
    b.bytes = want;
    return b.ptr;
}

void *pinned_get(jet_context *ctx, size_t bytes)
{
    if (ctx->pinned && ctx->pinned_bytes >= bytes) return ctx->pinned;
    void *p = nullptr;
    const size_t want = std::max(bytes + bytes / 4, (size_t)4096);
    if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    ctx->pinned = p;
    ctx->pinned_bytes = want;
    return p;
}

static int64_t balance_limit(int64_t W, int k, int lambda_ppm)
{
    return (int64_t)(((__int128)W * (1000000 + (__int128)lambda_ppm)) / ((__int128)k * 1000000));
}
static int64_t deadzone_sigma(int64_t W, int k, int64_t o, int div)
{
    const int64_t ceil_avg = (W + k - 1) / k;
    const int64_t slack = o - ceil_avg;
    if (slack <= 0) return o;
    if (slack < div) return o - 1;
    return o - slack / div;
}

#define JET_TRY(expr)                                      \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return hip_status(ctx, e_);  \
    } while (0)

// Up to this k the small-row role runs with 4 lanes per vertex (64 tables of
// k + 1 ints per block fit in 32 KiB): twice the vertices in flight per wave.
constexpr int K_G4 = 120;

// LDS of one compute unit (gfx950).
constexpr size_t LDS_PER_CU = 160 * 1024;

// Per-part candidate bounds (int64) and B flags of the small-row loss
// kernel, plus 4 bytes of alignment slack.
static size_t rb_cache_lds(int k) { return (size_t)k * 9 + 4; }

// Dynamic LDS of the wide small-row kernels (groups of 8 lanes), without the
// block histogram.
static size_t rb_s2_lds(int k) { return (BLOCK / 8) * (size_t)(k + 1) * 4 + BLOCK * 4; }

// Dynamic LDS of the loss kernel of a role (tables and queue), without the
// block histogram.
static size_t rb_role_lds(int role, int k)
{
    const size_t st = (size_t)(k + 1) * 4;
    if (role == 1) return (BLOCK / (k <= K_G4 ? 4 : 8)) * st + BLOCK * 4;
    if (role == 2) return (BLOCK / 64) * st + BLOCK * 4;
    if (role == 3) return (size_t)k * 4;
    return 0;
}

struct Plan {
    KArgs tab;    // LDS-table kernels (gain, loss)
    KArgs plain;  // afterburner, cut delta and the flat kernels
    int G;
    int grid_tab, grid_plain, grid_rbtab;
    size_t lds_tab;
    int grid_flat, grid_tile, grid_hist;
    int grid_lch;  // chunk kernels (0: no chunked rows)
    bool hist_fused;  // the loss kernels build the histogram (one graph, LDS room)
    bool cut_fused;   // the tile-sum blocks find the cut-off slots (one graph)
    bool loss_cache;  // the small-row loss kernel keeps per-part bounds in LDS (one graph)
    bool split_rows;  // one large graph, small class only: gain and loss in launches of their own
    int grid_lfin, nL;
    int grid_v;              // grid of the list-building kernels
    int32_t *blkcnt, *lcnt;  // their scratch
    int32_t *bins;
    bool hist_lds;
    // persistent connectivity table (one graph, JET_F_CONN_TABLE)
    bool table;
    int grid_tsmall, grid_tlarge;  // row scans and updates: small classes / medium and long rows
    int grid_tb[4];                // table build, per role (1, 2, 3)
    size_t lds_tb[4];
    bool small_g8 = false;         // batch: groups of 8 lanes for small rows even where k allows 4
};

static int div_up(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

int row_marks(jet_context *ctx, const int64_t *xadj, int n, int64_t nnz, int32_t **mark, int64_t *nmark,
              hipStream_t s)
{
    const int64_t nm = nnz / MARK + 1;
    int32_t *m = (int32_t *)ws_get(ctx, WS_RMARK, sizeof(int32_t) * (size_t)nm);
    if (!m) return JET_ENOMEM;
    k_row_marks<<<std::max(1, std::min(div_up(nm, BLOCK), ctx->num_cu)), BLOCK, 0, s>>>(xadj, n, nm, m);
    *mark = m;
    *nmark = nm;
    return JET_OK;
}

static void plan_roles(const jet_context *ctx, const KArgs &a, const int32_t *cnt, Plan &pl)
{
    const int maxb = ctx->num_cu * 8;
    const bool chunked = a.nlch > 0;  // L rows go to the chunk kernels
    // LDS-table kernels: the small-row role keeps 32 or 64 tables of k ints,
    // the wave role 4, the block role 1; larger k moves classes to roles with
    // fewer tables so a block stays within 64 KiB of LDS.
    KArgs t = a;
    t.tmap[0] = 0;
    const int k = a.k;
    if (k <= 495) { t.tmap[CLS_S] = 1; t.tmap[CLS_S2] = 1; t.tmap[CLS_M] = 2; t.tmap[CLS_L] = 3; }
    else if (k <= 4031) { t.tmap[CLS_S] = 2; t.tmap[CLS_S2] = 2; t.tmap[CLS_M] = 2; t.tmap[CLS_L] = 3; }
    else { t.tmap[CLS_S] = 3; t.tmap[CLS_S2] = 3; t.tmap[CLS_M] = 3; t.tmap[CLS_L] = 3; }
    if (chunked) t.tmap[CLS_L] = 0;
    int64_t role_cnt[4] = {0, 0, 0, 0};
    for (int c = 1; c < NCLS; c++) role_cnt[t.tmap[c]] += cnt[c];
    t.gS = t.tmap[CLS_S] == 1 ? std::min(div_up(cnt[CLS_S], BLOCK / 8), maxb) : 0;
    t.gS2 = t.tmap[CLS_S2] == 1 ? std::min(div_up(cnt[CLS_S2], BLOCK / 8), maxb) : 0;
    // one graph with every vertex in the small class (a mesh's finest levels):
    // its class list is the identity and is not read
    t.sident = a.vg == nullptr && cnt[CLS_S] == a.n ? 1 : 0;
    t.gM = std::min(div_up(role_cnt[2], BLOCK / 64), maxb);
    t.gL = std::min((int)role_cnt[3], maxb);
    t.gZ = std::min(div_up(cnt[0], BLOCK), maxb);
    size_t lds = 0;
    if (t.gS) lds = std::max(lds, (size_t)(BLOCK / 8) * k * 4);
    if (t.gM) lds = std::max(lds, (size_t)(BLOCK / 64) * k * 4);
    if (t.gL) lds = std::max(lds, (size_t)k * 4);
    pl.lds_tab = lds;
    pl.grid_tab = t.gS + t.gS2 + t.gM + t.gL;
    pl.grid_rbtab = t.gS + t.gS2 + t.gM + t.gL + t.gZ;
    // plain row kernels: roles follow the classes directly
    KArgs p = a;
    p.tmap[CLS_Z] = 0; p.tmap[CLS_S] = 1; p.tmap[CLS_S2] = 1; p.tmap[CLS_M] = 2; p.tmap[CLS_L] = 3;
    p.gS = std::min(div_up(cnt[CLS_S] + cnt[CLS_S2], BLOCK / 8), maxb);
    p.sident = t.sident;
    p.gM = std::min(div_up(cnt[CLS_M], BLOCK / 64), maxb);
    p.gL = chunked ? 0 : std::min(cnt[CLS_L], maxb);
    p.gZ = std::min(div_up(cnt[CLS_Z], BLOCK), maxb);
    pl.grid_plain = p.gS + p.gM + p.gL + p.gZ;
    pl.tab = t;
    pl.plain = p;
    pl.hist_lds = a.vg == nullptr && (size_t)a.k * NSLOT * 4 <= 65536;
    // The loss kernels keep a block histogram only where it costs no
    // occupancy: every block of each role stays resident at once.
    pl.hist_fused = a.vg == nullptr;
    // (the small-row role: one launch of gS + gS2 blocks when both classes have rows)
    const int rgrid[5] = {0, t.gS + t.gS2, t.gM, t.gL, t.gZ};
    for (int r = 1; r <= 4; r++) {
        const size_t base = (r == 1 && !t.gS) ? rb_s2_lds(k) : rb_role_lds(r, k);
        const size_t per = base + (size_t)k * NSLOT * 4;
        if (per > 65536 || (size_t)div_up(rgrid[r], ctx->num_cu) * per > LDS_PER_CU) pl.hist_fused = false;
    }
    pl.cut_fused = a.vg == nullptr && k <= 1024;
    {
        const size_t extra = (pl.hist_fused ? (size_t)k * NSLOT * 4 : 0) + rb_cache_lds(k);
        const size_t per = (t.gS ? rb_role_lds(1, k) : rb_s2_lds(k)) + extra;
        pl.loss_cache = a.vg == nullptr && k <= 1024 && per <= 65536 &&
                        (size_t)div_up(t.gS + t.gS2, ctx->num_cu) * per <= LDS_PER_CU;
    }
    // A large graph whose rows are all in the small class (a mesh's finest
    // levels): the gain pass is long enough that its own launch, with two
    // rows in flight per group, pays for the extra launch per iteration.
    pl.split_rows = a.vg == nullptr && t.gS && !t.gS2 && a.n >= (1 << 18);
    pl.table = a.toff != nullptr;
    if (pl.table) {
        // row scans build no block histogram; no split small-row launches
        pl.hist_fused = false;
        pl.split_rows = false;
        pl.grid_tsmall = std::min(std::max(div_up(cnt[CLS_S] + cnt[CLS_S2], BLOCK / 8), div_up(cnt[CLS_Z], BLOCK)), maxb);
        pl.grid_tlarge = std::min(div_up(cnt[CLS_M] + cnt[CLS_L], BLOCK / 64), maxb);
        int64_t rows[4] = {0, 0, 0, 0};
        for (int c = CLS_S; c <= CLS_L; c++) rows[(c == CLS_L || t.tmap[c] == 0) ? 3 : t.tmap[c]] += cnt[c];
        pl.grid_tb[1] = rows[1] ? std::min(div_up(rows[1], BLOCK / 8), maxb) : 0;
        pl.grid_tb[2] = rows[2] ? std::min(div_up(rows[2], BLOCK / 64), maxb) : 0;
        pl.grid_tb[3] = rows[3] ? (int)std::min<int64_t>(rows[3], maxb) : 0;
        pl.lds_tb[1] = (size_t)(BLOCK / 8) * (k + 1) * 4;
        pl.lds_tb[2] = (size_t)(BLOCK / 64) * (k + 1) * 4;
        pl.lds_tb[3] = (size_t)k * 4;
    }
    pl.grid_hist = std::max(1, std::min(div_up(a.n, BLOCK), ctx->num_cu * 2));
    pl.grid_flat = std::max(1, std::min(div_up(a.n, BLOCK), ctx->num_cu * 2));
    pl.grid_tile = std::max(1, std::min(a.ntile, ctx->num_cu * 8));
    pl.grid_lch = chunked ? std::max(1, std::min(a.nlch, maxb)) : 0;
    pl.nL = cnt[CLS_L];
    pl.grid_lfin = chunked ? std::max(1, std::min(div_up(pl.nL, BLOCK / 64), maxb)) : 0;
}


template <bool B>
static void launch_gain_t(const Plan &pl, hipStream_t s, bool small = true)
{
    const KArgs &t = pl.tab;
    const size_t st = (size_t)(t.k + 1) * 4;
    // small rows: one launch for both small classes when both are present
    if (!small) {
    } else if (t.gS && t.gS2) {
        const int g = t.gS + t.gS2;
        if (t.k <= K_G4 && !pl.small_g8) k_gain<B, 1, 4, 8, NCLS><<<g, BLOCK, (BLOCK / 4) * st + BLOCK * 4, s>>>(t, g);
        else k_gain<B, 1, 8, 4, NCLS><<<g, BLOCK, (BLOCK / 8) * st + BLOCK * 4, s>>>(t, g);
    } else if (t.gS) {
        if (t.k <= K_G4 && !pl.small_g8) k_gain<B, 1, 4><<<t.gS, BLOCK, (BLOCK / 4) * st + BLOCK * 4, s>>>(t, t.gS);
        else k_gain<B, 1, 8><<<t.gS, BLOCK, (BLOCK / 8) * st + BLOCK * 4, s>>>(t, t.gS);
    } else if (t.gS2) {
        k_gain<B, 1, 8, 8, CLS_S2><<<t.gS2, BLOCK, rb_s2_lds(t.k), s>>>(t, t.gS2);
    }
    if (t.gM) k_gain<B, 2><<<t.gM, BLOCK, (BLOCK / 64) * st + BLOCK * 4, s>>>(t, t.gM);
    if (t.gL) k_gain<B, 3><<<t.gL, BLOCK, (size_t)t.k * 4, s>>>(t, t.gL);
    if (pl.grid_lch) {
        k_lconn<B, false><<<pl.grid_lch, BLOCK, (size_t)t.k * 4, s>>>(t, HIST_NONE);
        k_lgain_fin<B><<<pl.grid_lfin, BLOCK, 0, s>>>(t);
    }
}

// Afterburner and the rebalancing tile sums in one launch (each pass exits
// at once in iterations of the other kind), then the long-row afterburner.
template <bool B>
static void launch_after_t(const Plan &pl, hipStream_t s)
{
    const KArgs &p = pl.plain;
    const size_t lds = (size_t)p.k * 4 * (pl.cut_fused ? 2 : 1);
    k_after_tsum<B><<<pl.grid_plain + pl.grid_tile, BLOCK, lds, s>>>(p, pl.grid_plain, pl.cut_fused ? 1 : 0);
    if (pl.grid_lch) {
        k_lafter<B><<<pl.grid_lch, BLOCK, 0, s>>>(p);
        k_lafter_fin<B><<<std::max(1, div_up(pl.nL, BLOCK)), BLOCK, 0, s>>>(p);
    }
}

template <bool B>
static void launch_rb_loss_t(const Plan &pl, hipStream_t s, bool small = true)
{
    const KArgs &t = pl.tab;
    const int hm = pl.hist_fused ? HIST_LDS : HIST_NONE;
    const size_t hb = pl.hist_fused ? (size_t)t.k * NSLOT * 4 : 0;
    const size_t cb = pl.loss_cache ? rb_cache_lds(t.k) : 0;
    if (!small) {
    } else if (t.gS && t.gS2) {
        const size_t l1 = rb_role_lds(1, t.k) + hb + cb;
        const int g = t.gS + t.gS2;
        const bool g4 = t.k <= K_G4 && !pl.small_g8;
        if (pl.loss_cache) {
            if (g4) k_rb_loss<B, 1, 4, 8, true, NCLS><<<g, BLOCK, l1, s>>>(t, g, hm);
            else k_rb_loss<B, 1, 8, 4, true, NCLS><<<g, BLOCK, l1, s>>>(t, g, hm);
        } else {
            if (g4) k_rb_loss<B, 1, 4, 8, false, NCLS><<<g, BLOCK, l1, s>>>(t, g, hm);
            else k_rb_loss<B, 1, 8, 4, false, NCLS><<<g, BLOCK, l1, s>>>(t, g, hm);
        }
    } else if (t.gS) {
        const size_t l1 = rb_role_lds(1, t.k) + hb + cb;
        const bool g4 = t.k <= K_G4 && !pl.small_g8;
        if (pl.loss_cache) {
            if (g4) k_rb_loss<B, 1, 4, 8, true><<<t.gS, BLOCK, l1, s>>>(t, t.gS, hm);
            else k_rb_loss<B, 1, 8, 4, true><<<t.gS, BLOCK, l1, s>>>(t, t.gS, hm);
        } else {
            if (g4) k_rb_loss<B, 1, 4><<<t.gS, BLOCK, l1, s>>>(t, t.gS, hm);
            else k_rb_loss<B, 1, 8><<<t.gS, BLOCK, l1, s>>>(t, t.gS, hm);
        }
    } else if (t.gS2) {
        const size_t l2 = rb_s2_lds(t.k) + hb + cb;
        if (pl.loss_cache) k_rb_loss<B, 1, 8, 8, true, CLS_S2><<<t.gS2, BLOCK, l2, s>>>(t, t.gS2, hm);
        else k_rb_loss<B, 1, 8, 8, false, CLS_S2><<<t.gS2, BLOCK, l2, s>>>(t, t.gS2, hm);
    }
    if (t.gM) k_rb_loss<B, 2><<<t.gM, BLOCK, rb_role_lds(2, t.k) + hb, s>>>(t, t.gM, hm);
    if (t.gL) k_rb_loss<B, 3><<<t.gL, BLOCK, rb_role_lds(3, t.k) + hb, s>>>(t, t.gL, hm);
    if (t.gZ) k_rb_loss<B, 4><<<t.gZ, BLOCK, rb_role_lds(4, t.k) + hb, s>>>(t, t.gZ, hm);
    if (pl.grid_lch) {
        const int lh = pl.hist_fused ? HIST_GLOBAL : HIST_NONE;
        k_lconn<B, true><<<pl.grid_lch, BLOCK, (size_t)t.k * 4, s>>>(t, lh);
        k_lrb_fin<B><<<pl.grid_lfin, BLOCK, 0, s>>>(t, lh);
    }
}

// Histogram and cut-off slots where the loss and tile-sum passes do not
// find them themselves.
template <bool B>
static void launch_rb_cutoff_t(const Plan &pl, hipStream_t s)
{
    const KArgs &p = pl.plain;
    if (!pl.hist_fused) k_rb_hist<B><<<pl.grid_hist, BLOCK, pl.hist_lds ? (size_t)p.k * NSLOT * 4 : 0, s>>>(p, pl.hist_lds);
    if (!pl.cut_fused) k_rb_cutoff<<<pl.G, BLOCK, 0, s>>>(p);
}

// Ordered selection (split, mark) and the Jetrs cookie-cutter.
template <bool B>
static void launch_rb_select_t(const Plan &pl, hipStream_t s)
{
    const KArgs &p = pl.plain;
    k_rb_split<<<std::min(p.ktot, 1024), BLOCK, 0, s>>>(p);
    k_rb_mark<<<pl.grid_tile, BLOCK, 0, s>>>(p);
    k_rs_assign<<<pl.grid_tile, BLOCK, 0, s>>>(p);
}

// One graph: the small-row gain and loss passes in one launch (k_rows).
template <bool PC>
static void launch_rows_t(const Plan &pl, hipStream_t s)
{
    const KArgs &t = pl.tab;
    const int hm = pl.hist_fused ? HIST_LDS : HIST_NONE;
    const size_t extra = (pl.hist_fused ? (size_t)t.k * NSLOT * 4 : 0) + (PC ? rb_cache_lds(t.k) : 0);
    if (t.gS && t.gS2) {
        const int g = t.gS + t.gS2;
        if (t.k <= K_G4) k_rows<4, 8, PC, NCLS><<<g, BLOCK, rb_role_lds(1, t.k) + extra, s>>>(t, g, hm);
        else k_rows<8, 4, PC, NCLS><<<g, BLOCK, rb_role_lds(1, t.k) + extra, s>>>(t, g, hm);
    } else if (t.gS) {
        if (t.k <= K_G4) k_rows<4, 8, PC, CLS_S><<<t.gS, BLOCK, rb_role_lds(1, t.k) + extra, s>>>(t, t.gS, hm);
        else k_rows<8, 4, PC, CLS_S><<<t.gS, BLOCK, rb_role_lds(1, t.k) + extra, s>>>(t, t.gS, hm);
    } else if (t.gS2) {
        k_rows<8, 8, PC, CLS_S2><<<t.gS2, BLOCK, rb_s2_lds(t.k) + extra, s>>>(t, t.gS2, hm);
    }
}

// Table mode: the row scans (gain, loss), the update passes, the builds.
static void launch_tab_scan(const Plan &pl, hipStream_t s, bool rb)
{
    const int g = pl.grid_tsmall + pl.grid_tlarge;
    if (!g) return;
    if (rb) k_tab_scan<true><<<g, BLOCK, 0, s>>>(pl.tab, pl.grid_tsmall);
    else k_tab_scan<false><<<g, BLOCK, 0, s>>>(pl.tab, pl.grid_tsmall);
}

static void launch_tab_build(const Plan &pl, hipStream_t s, int setup)
{
    if (pl.grid_tb[1]) k_tab_build<1><<<pl.grid_tb[1], BLOCK, pl.lds_tb[1], s>>>(pl.tab, setup);
    if (pl.grid_tb[2]) k_tab_build<2><<<pl.grid_tb[2], BLOCK, pl.lds_tb[2], s>>>(pl.tab, setup);
    if (pl.grid_tb[3]) k_tab_build<3><<<pl.grid_tb[3], BLOCK, pl.lds_tb[3], s>>>(pl.tab, setup);
}

static void launch_iteration_table(const Plan &pl, hipStream_t s, hipEvent_t ev_a, hipEvent_t ev_b)
{
    const KArgs &p = pl.plain;
    if (ev_a) (void)hipEventRecord(ev_a, s);
    launch_tab_scan(pl, s, false);
    if (ev_b) (void)hipEventRecord(ev_b, s);
    launch_tab_scan(pl, s, true);
    launch_rb_cutoff_t<false>(pl, s);
    launch_after_t<false>(pl, s);
    launch_rb_select_t<false>(pl, s);
    if (pl.grid_plain) k_dcut<false><<<pl.grid_plain, BLOCK, 0, s>>>(p);
    if (pl.grid_lch) k_ldcut<false><<<pl.grid_lch, BLOCK, 0, s>>>(p);
    const int gu = pl.grid_tsmall + pl.grid_tlarge;
    if (gu) k_tab_update<<<gu, BLOCK, 0, s>>>(p, pl.grid_tsmall);
    k_apply<false><<<pl.grid_flat, BLOCK, (size_t)p.k * 4, s>>>(p);
    launch_tab_build(pl, s, 0);
    k_ctl_end<<<pl.G, BLOCK, 0, s>>>(p);
}

template <bool B>
static void launch_iteration_t(const Plan &pl, hipStream_t s, hipEvent_t ev_a, hipEvent_t ev_b)
{
    if (!B && pl.table) {
        launch_iteration_table(pl, s, ev_a, ev_b);
        return;
    }
    const KArgs &p = pl.plain;
    if (ev_a) (void)hipEventRecord(ev_a, s);
    const bool split = !B && pl.split_rows;
    if (!B && !split) {
        if (pl.loss_cache) launch_rows_t<true>(pl, s);
        else launch_rows_t<false>(pl, s);
    }
    launch_gain_t<B>(pl, s, B || split);
    if (ev_b) (void)hipEventRecord(ev_b, s);
    launch_rb_loss_t<B>(pl, s, B || split);
    launch_rb_cutoff_t<B>(pl, s);
    launch_after_t<B>(pl, s);
    launch_rb_select_t<B>(pl, s);
    if (pl.grid_plain) k_dcut<B><<<pl.grid_plain, BLOCK, 0, s>>>(p);
    if (pl.grid_lch) k_ldcut<B><<<pl.grid_lch, BLOCK, 0, s>>>(p);
    k_apply<B><<<pl.grid_flat, BLOCK, B ? 0 : (size_t)p.k * 4, s>>>(p);
    k_ctl_end<<<pl.G, BLOCK, 0, s>>>(p);
}

static bool batched(const Plan &pl) { return pl.plain.vg != nullptr; }

static void launch_gain(const Plan &pl, hipStream_t s)
{
    if (batched(pl)) launch_gain_t<true>(pl, s);
    else if (pl.table) launch_tab_scan(pl, s, false);
    else launch_gain_t<false>(pl, s);
}
static void launch_after(const Plan &pl, hipStream_t s)
{
    if (batched(pl)) launch_after_t<true>(pl, s);
    else launch_after_t<false>(pl, s);
}
static void launch_rb_loss(const Plan &pl, hipStream_t s)
{
    if (batched(pl)) launch_rb_loss_t<true>(pl, s);
    else if (pl.table) launch_tab_scan(pl, s, true);
    else launch_rb_loss_t<false>(pl, s);
}
static void launch_rb_cutoff(const Plan &pl, hipStream_t s)
{
    if (batched(pl)) launch_rb_cutoff_t<true>(pl, s);
    else launch_rb_cutoff_t<false>(pl, s);
}
static void launch_rb_select(const Plan &pl, hipStream_t s)
{
    if (batched(pl)) launch_rb_select_t<true>(pl, s);
    else launch_rb_select_t<false>(pl, s);
}
static void launch_iteration(const Plan &pl, hipStream_t s, hipEvent_t ev_a = nullptr, hipEvent_t ev_b = nullptr)
{
    if (batched(pl)) launch_iteration_t<true>(pl, s, ev_a, ev_b);
    else launch_iteration_t<false>(pl, s, ev_a, ev_b);
}

static void set_it(Plan &pl, int it)
{
    pl.tab.it = it;
    pl.plain.it = it;
}

template <bool B>
static void set_lds_limits_t()
{
    (void)hipFuncSetAttribute((const void *)k_gain<B, 1, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_gain<B, 1, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_gain<B, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_gain<B, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_rb_loss<B, 1, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_rb_loss<B, 1, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_rb_loss<B, 1, 4, 8, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              65536);
    (void)hipFuncSetAttribute((const void *)k_rb_loss<B, 1, 8, 4, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              65536);
    (void)hipFuncSetAttribute((const void *)k_rb_loss<B, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_rb_loss<B, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_rb_loss<B, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_gain<B, 1, 8, 8, CLS_S2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              65536);
    (void)hipFuncSetAttribute((const void *)k_gain<B, 1, 4, 8, NCLS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              65536);
    (void)hipFuncSetAttribute((const void *)k_gain<B, 1, 8, 4, NCLS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              65536);
    (void)hipFuncSetAttribute((const void *)k_rb_loss<B, 1, 4, 8, true, NCLS>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_rb_loss<B, 1, 8, 4, true, NCLS>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_rb_loss<B, 1, 4, 8, false, NCLS>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_rb_loss<B, 1, 8, 4, false, NCLS>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_rb_loss<B, 1, 8, 8, true, CLS_S2>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_rb_loss<B, 1, 8, 8, false, CLS_S2>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_apply<B>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_rb_hist<B>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_after_tsum<B>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_lconn<B, false>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_lconn<B, true>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
}

template <bool PC>
static void set_lds_limits_rows()
{
    (void)hipFuncSetAttribute((const void *)k_rows<4, 8, PC, NCLS>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_rows<8, 4, PC, NCLS>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_rows<4, 8, PC, CLS_S>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_rows<8, 4, PC, CLS_S>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_rows<8, 8, PC, CLS_S2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              65536);
}

// Once per process, before any launch needing more than the default dynamic
// LDS (call_once: serving lanes set up concurrently, and none may launch
// before the limits are in place).
static void set_lds_limits()
{
    static std::once_flag once;
    std::call_once(once, [] {
        set_lds_limits_t<false>();
        set_lds_limits_t<true>();
        set_lds_limits_rows<false>();
        set_lds_limits_rows<true>();
        (void)hipFuncSetAttribute((const void *)k_init_vertices, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
        (void)hipFuncSetAttribute((const void *)k_tab_build<1>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
        (void)hipFuncSetAttribute((const void *)k_tab_build<2>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
        (void)hipFuncSetAttribute((const void *)k_tab_build<3>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    });
}

static int check_params(const jet_csr *g, const jet_params *prm)
{
    if (!g || !prm) return JET_EINVAL;
    if (prm->k < 1 || prm->lambda_ppm < 0 || prm->c_den < 0 || prm->c_num < 0 || prm->phi_den < 0 ||
        prm->phi_num < 0 || prm->stall_limit < 0 || prm->deadzone_div < 0 || prm->max_iters < 0 ||
        prm->weak_rebalance_iters < -1 || prm->level < 0)
        return JET_EINVAL;
    if (prm->c_den > 0 && prm->c_num > prm->c_den * 64) return JET_EINVAL;
    if (prm->k > KMAX) return JET_ELIMIT;
    if (g->n < 0 || g->nnz < 0) return JET_EGRAPH;
    if (g->n > 0 && (!g->xadj)) return JET_EINVAL;
    if (g->nnz > 0 && !g->adjncy) return JET_EINVAL;
    return JET_OK;
}

// Host-side full CSR check (JET_F_VALIDATE): symmetric with equal weights,
// no duplicates, no self-loops, ids in range.
int validate_full_csr(jet_context *ctx, const jet_csr *g, hipStream_t s)
{
    const int n = g->n;
    const int64_t nnz = g->nnz;
    std::vector<int64_t> xadj(n + 1);
    std::vector<int32_t> adj(nnz), ew(nnz, 1);
    JET_TRY(hipMemcpyAsync(xadj.data(), g->xadj, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, s));
    if (nnz) JET_TRY(hipMemcpyAsync(adj.data(), g->adjncy, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, s));
    if (nnz && g->adjwgt) JET_TRY(hipMemcpyAsync(ew.data(), g->adjwgt, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, s));
    JET_TRY(stream_wait(ctx, s));
    if (xadj[0] != 0 || xadj[n] != nnz) return JET_EGRAPH;
    std::vector<std::pair<uint64_t, int32_t>> kw(nnz), rkw(nnz);
    for (int v = 0; v < n; v++) {
        if (xadj[v + 1] < xadj[v]) return JET_EGRAPH;
        for (int64_t e = xadj[v]; e < xadj[v + 1]; e++) {
            const int u = adj[e];
            if (u < 0 || u >= n || u == v || ew[e] < 1) return JET_EGRAPH;
            kw[e] = {((uint64_t)(uint32_t)v << 32) | (uint32_t)u, ew[e]};
            rkw[e] = {((uint64_t)(uint32_t)u << 32) | (uint32_t)v, ew[e]};
        }
    }
    std::sort(kw.begin(), kw.end());
    std::sort(rkw.begin(), rkw.end());
    for (int64_t e = 0; e < nnz; e++) {
        if (e > 0 && kw[e].first == kw[e - 1].first) return JET_EGRAPH;
        if (kw[e] != rkw[e]) return JET_EGRAPH;
    }
    return JET_OK;
}

struct DebugOut {
    int64_t *F = nullptr, *cs = nullptr, *F2 = nullptr, *loss = nullptr;
    int32_t *pd = nullptr, *slot = nullptr;
};

// Controller configuration of one graph from its parameters.
static Ctl make_ctl(const jet_params *prm, int n)
{
    Ctl hc;
    memset(&hc, 0, sizeof(hc));
    hc.n = n;
    hc.k = prm->k;
    hc.stall_limit = prm->stall_limit > 0 ? prm->stall_limit : 12;
    hc.bmax = prm->weak_rebalance_iters == 0 ? 2 : (prm->weak_rebalance_iters < 0 ? 0 : prm->weak_rebalance_iters);
    hc.max_iters = prm->max_iters;
    if (prm->c_den > 0) {
        hc.c_num = prm->c_num;
        hc.c_den = prm->c_den;
    } else {
        hc.c_num = prm->level == 0 ? 1 : 3;
        hc.c_den = 4;
    }
    hc.phi_num = prm->phi_num > 0 ? prm->phi_num : 999;
    hc.phi_den = prm->phi_den > 0 ? prm->phi_den : 1000;
    hc.level = prm->level;
    hc.seed = prm->seed;
    hc.lambda_ppm = prm->lambda_ppm;
    hc.deadzone_div = prm->deadzone_div > 0 ? prm->deadzone_div : 10;
    hc.flags = (int32_t)prm->flags;
    return hc;
}

// One refinement launch over G graphs laid out as a union (for G = 1 the
// caller's own graph and arrays).
struct Launch {
    int G = 1;
    jet_csr u;                                               // union CSR
    const int32_t *vg = nullptr, *pg = nullptr, *tg = nullptr;  // device maps (NULL for one graph)
    const int32_t *part_in = nullptr;                        // P_0
    int32_t *best = nullptr;                                 // P_best (may be part_in)
    std::vector<Ctl> hc;                                     // per graph: configuration in, final state out
    int ktot = 0, kmax = 0, ntile = 0;
    int64_t tsum_cap = 0;
    jet_trace_rec *trace_dev = nullptr;
    // one graph whose P_0 is a projection: its cut, known from the coarser
    // level (>= 0), replaces the set-up edge pass
    int64_t cut0 = -1;
};

// Fills the workspace and the controllers, runs the set-up passes and
// returns the launch plan. Per-graph offsets (voff, poff, t0, ntiles,
// rowbase, trace_off, trace_cap) must already be in L.hc.
static int setup(jet_context *ctx, Launch &L, Plan &pl, hipStream_t s, const DebugOut *dbg)
{
    set_lds_limits();
    const int G = L.G;
    const int n = L.u.n;
    KArgs a;
    memset(&a, 0, sizeof(a));
    a.n = n;
    a.k = L.kmax;
    a.ngraph = G;
    a.ktot = L.ktot;
    a.xadj = L.u.xadj;
    a.adj = L.u.adjncy;
    a.vw = L.u.vwgt;
    a.ew = L.u.adjwgt;
    a.vg = L.vg;
    a.pg = L.pg;
    a.tg = L.tg;
    const size_t nn = (size_t)std::max(n, 1);
    const size_t kt = (size_t)L.ktot;
    a.P = (uint16_t *)ws_get(ctx, WS_P, nn * 2);
    const bool part8 = ctx->part8 && L.kmax <= 256;
    a.P8 = part8 ? (uint8_t *)ws_get(ctx, WS_P8, nn) : nullptr;
    a.mq = ws_get(ctx, WS_MQ, nn * (part8 ? 2 : 4));
    a.rq = part8 ? (uint32_t *)ws_get(ctx, WS_RQ, nn * 4) : nullptr;
    a.Fx = part8 ? (int32_t *)ws_get(ctx, WS_FX, nn * 4) : nullptr;
    if ((part8 && (!a.P8 || !a.rq || !a.Fx)) || !a.mq) return JET_ENOMEM;
    a.rec = (int2 *)ws_get(ctx, WS_REC, nn * 8);
    a.dest = (int32_t *)ws_get(ctx, WS_DEST, nn * 4);
    a.lock = (int32_t *)ws_get(ctx, WS_LOCK, nn * 4);
    a.slot = (uint8_t *)ws_get(ctx, WS_SLOT, nn);
    a.rbd = (int32_t *)ws_get(ctx, WS_RBD, nn * 4);
    a.rsev = (uint8_t *)ws_get(ctx, WS_RSEV, nn);
    int32_t *bins = (int32_t *)ws_get(ctx, WS_BIN, nn * 4);
    a.bins = bins;
    a.bstat = (int64_t *)ws_get(ctx, WS_BSTAT, sizeof(int64_t) * NSTAT * NSHARD * (size_t)G);
    a.cnt = (int32_t *)ws_get(ctx, WS_CNT, sizeof(int32_t) * (CNT_N + 2));
    a.ctl = (Ctl *)ws_get(ctx, WS_CTL, sizeof(Ctl) * (size_t)G);
    int64_t *p64 = (int64_t *)ws_get(ctx, WS_PART64, sizeof(int64_t) * (4 * kt + G + 8));
    int32_t *p32 = (int32_t *)ws_get(ctx, WS_PART32, sizeof(int32_t) * (3 * kt + 8));
    uint8_t *p8 = (uint8_t *)ws_get(ctx, WS_PART8, 2 * kt + 16);
    a.hist = (int64_t *)ws_get(ctx, WS_HIST, sizeof(int64_t) * kt * NSLOT);
    a.ntile = L.ntile;
    a.tsum = (int32_t *)ws_get(ctx, WS_TSUM, sizeof(int32_t) * (size_t)std::max<int64_t>(L.tsum_cap, 1));
    a.esum = (int64_t *)ws_get(ctx, WS_ESUM, sizeof(int64_t) * (size_t)std::max(L.ntile, 1));
    a.kinds = (int8_t *)ws_get(ctx, WS_KINDS, KIND_LOG);
    const int grid_v = std::max(1, std::min(div_up(n, BLOCK), ctx->num_cu * 4));
    int32_t *blkcnt = (int32_t *)ws_get(ctx, WS_BLKCNT, sizeof(int32_t) * ((size_t)grid_v + 1) * NCLS);
    char *pin = (char *)pinned_get(ctx, 4096 + sizeof(Ctl) * (size_t)G);
    if (!a.P || !a.rec || !a.dest || !a.lock || !a.slot || !a.rbd || !a.rsev || !bins || !a.bstat || !a.cnt ||
        !a.ctl || !p64 || !p32 || !p8 || !a.hist || !a.tsum || !a.esum || !a.kinds || !blkcnt || !pin)
        return JET_ENOMEM;
    a.w = p64;
    a.wbest = p64 + kt;
    a.resid = p64 + 2 * kt;
    a.capstart = p64 + 3 * kt;
    a.Blist = p32;
    a.sstar = p32 + kt;
    a.vthr = p32 + 2 * kt;
    a.isA = p8;
    a.isB = p8 + kt;
    a.best = L.best;
    a.trace = L.trace_dev;
    if (dbg) {
        a.dbg_F = dbg->F;
        a.dbg_cs = dbg->cs;
        a.dbg_F2 = dbg->F2;
        a.dbg_loss = dbg->loss;
        a.dbg_pd = dbg->pd;
        a.dbg_slot = dbg->slot;
    }
    Ctl *hcs = (Ctl *)(pin + 4096);
    memcpy(hcs, L.hc.data(), sizeof(Ctl) * G);
    JET_TRY(hipMemcpyAsync(a.ctl, hcs, sizeof(Ctl) * G, hipMemcpyHostToDevice, s));
    JET_TRY(hipMemsetAsync(a.w, 0, sizeof(int64_t) * kt, s));
    JET_TRY(hipMemsetAsync(a.bstat, 0, sizeof(int64_t) * NSTAT * NSHARD * (size_t)G, s));
    JET_TRY(hipMemsetAsync(a.cnt, 0, sizeof(int32_t) * (CNT_N + 2), s));
    if (n > 0) k_init_vertices<<<grid_v, BLOCK, a.vg ? 0 : (size_t)a.k * 4, s>>>(a, L.part_in, blkcnt);
    const bool known_cut = L.G == 1 && L.cut0 >= 0;
    if (L.u.nnz > 0 && !known_cut) {
        const int grid_e = std::max(1, std::min(div_up(L.u.nnz, MARK), ctx->num_cu * 8));
        int32_t *mark = nullptr;
        int64_t nmark = 0;
        const int rs = row_marks(ctx, L.u.xadj, n, L.u.nnz, &mark, &nmark, s);
        if (rs) return rs;
        k_init_edges<<<grid_e, BLOCK, 0, s>>>(a, L.u.nnz, mark, nmark);
    }
    k_bin_scan<<<1, BLOCK, 0, s>>>(blkcnt, grid_v);
    const int32_t *ctot = blkcnt + (size_t)grid_v * NCLS;  // class totals on the device
    if (n > 0) k_fill_bins<<<grid_v, BLOCK, 0, s>>>(a, blkcnt, bins);
    // chunks of the long (L class) rows: count and scan now, list after the sync
    int32_t *lcnt = (int32_t *)ws_get(ctx, WS_LCNT, sizeof(int32_t) * (nn + 1));
    if (!lcnt) return JET_ENOMEM;
    int32_t *lmeta = a.cnt + CNT_N;  // total chunk count
    if (n > 0) {
        k_lchunk_count<<<grid_v, BLOCK, 0, s>>>(a.xadj, bins, ctot, lcnt);
        k_lchunk_scan<<<1, BLOCK, 0, s>>>(ctot, lcnt, lmeta);
    }
    k_init_reduce<<<G, 64, 0, s>>>(a);
    JET_TRY(hipGetLastError());
    int32_t *hcnt = (int32_t *)pin;             // CNT_N counts
    int32_t *htot = (int32_t *)(pin + 64);      // class totals
    int64_t *xends = (int64_t *)(pin + 128);    // first and last row offset (one graph)
    JET_TRY(hipMemcpyAsync(hcs, a.ctl, sizeof(Ctl) * G, hipMemcpyDeviceToHost, s));
    JET_TRY(hipMemcpyAsync(hcnt, a.cnt, sizeof(int32_t) * (CNT_N + 1), hipMemcpyDeviceToHost, s));
    JET_TRY(hipMemcpyAsync(htot, blkcnt + (size_t)grid_v * NCLS, sizeof(int32_t) * NCLS, hipMemcpyDeviceToHost, s));
    JET_TRY(hipMemcpyAsync(xends, L.u.xadj, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    JET_TRY(hipMemcpyAsync(xends + 1, L.u.xadj + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    JET_TRY(stream_wait(ctx, s));
    if (xends[0] != 0 || xends[1] != L.u.nnz || hcnt[1]) return JET_EGRAPH;
    for (int g = 0; g < G; g++)
        if (hcs[g].bad_part) return JET_EPART;
    if (known_cut) hcs[0].cut = L.cut0;
    // limits: total vertex weight below 2^31 (part weights, tile sums), and
    // every weighted degree below 2^31 (connectivities, gains, losses are
    // int32); the exact degree check runs only when the total edge weight
    // does not already bound them
    bool wide = false;
    for (int g = 0; g < G; g++) {
        if (hcs[g].wsum >= ((int64_t)1 << 31)) return JET_EOVERFLOW;
        if (hcs[g].ewsum >= ((int64_t)1 << 31)) wide = true;
    }
    if (wide && L.u.adjwgt) {
        unsigned long long *dmax = (unsigned long long *)ws_get(ctx, WS_WDEG, 16);
        if (!dmax) return JET_ENOMEM;
        JET_TRY(hipMemsetAsync(dmax, 0, 8, s));
        k_wdeg_max<<<std::max(1, std::min(div_up(n, BLOCK / 64), ctx->num_cu * 8)), BLOCK, 0, s>>>(
            L.u.xadj, L.u.adjwgt, n, dmax);
        JET_TRY(hipGetLastError());
        JET_TRY(hipMemcpyAsync(pin + 256, dmax, 8, hipMemcpyDeviceToHost, s));
        JET_TRY(stream_wait(ctx, s));
        if (*(const uint64_t *)(pin + 256) >= ((uint64_t)1 << 31)) return JET_EOVERFLOW;
    }
    for (int g = 0; g < G; g++) {
        Ctl &c = hcs[g];
        c.W = c.wsum;
        c.o = balance_limit(c.W, c.k, c.lambda_ppm);
        c.sigma = deadzone_sigma(c.W, c.k, c.o, c.deadzone_div);
    }
    JET_TRY(hipMemcpyAsync(a.ctl, hcs, sizeof(Ctl) * G, hipMemcpyHostToDevice, s));
    a.binoff[0] = 0;
    int32_t tot[NCLS];
    for (int c = 0; c < NCLS; c++) {
        tot[c] = htot[c];
        a.binoff[c + 1] = a.binoff[c] + tot[c];
    }
    // chunked long rows when the per-chunk connectivity rows fit in 512 MiB
    // (else the block role walks each long row alone)
    const int nL = tot[CLS_L];
    const int nch = hcnt[CNT_N];
    if (nL > 0 && nch > 0 && (size_t)nch * (size_t)L.kmax * 4 <= ((size_t)512 << 20)) {
        int2 *lch = (int2 *)ws_get(ctx, WS_LCH, sizeof(int2) * (size_t)nch);
        int32_t *gconn = (int32_t *)ws_get(ctx, WS_GCONN, sizeof(int32_t) * (size_t)nch * L.kmax);
        int32_t *ldone = (int32_t *)ws_get(ctx, WS_LDONE, sizeof(int32_t) * 2 * (size_t)nL);
        if (!lch || !gconn || !ldone) return JET_ENOMEM;
        JET_TRY(hipMemsetAsync(ldone, 0, sizeof(int32_t) * 2 * (size_t)nL, s));
        k_lchunk_fill<<<grid_v, BLOCK, 0, s>>>(ctot, lcnt, lch);
        a.lch = lch;
        a.lcoff = lcnt;
        a.nlch = nch;
        a.lstride = L.kmax;
        a.gconn = gconn;
        a.ldone = ldone;
        a.gf2 = ldone + nL;
    }
    // batch: work-queue counters of the row kernels (both banks clear)
    if (a.vg != nullptr) {
        a.wq = (int32_t *)ws_get(ctx, WS_WQ, sizeof(int32_t) * 2 * NQC);
        if (!a.wq) return JET_ENOMEM;
        JET_TRY(hipMemsetAsync(a.wq, 0, sizeof(int32_t) * 2 * NQC, s));
        a.wtile = 0;
    }
    // persistent connectivity table (one graph, JET_F_CONN_TABLE): row
    // offsets, then the rows built from P_0 once the roles are planned
    int64_t tslots = 0;
    if (a.vg == nullptr && (L.hc[0].flags & JET_F_CONN_TABLE) && n > 0) {
        int64_t *toff = (int64_t *)ws_get(ctx, WS_TOFF, sizeof(int64_t) * (nn + 1));
        int64_t *tblk = (int64_t *)ws_get(ctx, WS_TBLK, sizeof(int64_t) * ((size_t)grid_v + 1));
        if (!toff || !tblk) return JET_ENOMEM;
        k_toff_count<<<grid_v, BLOCK, 0, s>>>(a.xadj, n, a.k, tblk);
        k_toff_scan<<<1, BLOCK, 0, s>>>(tblk, grid_v);
        k_toff_fill<<<grid_v, BLOCK, 0, s>>>(a.xadj, n, a.k, tblk, toff);
        JET_TRY(hipMemcpyAsync(pin + 264, tblk + grid_v, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        JET_TRY(stream_wait(ctx, s));
        tslots = *(const int64_t *)(pin + 264);
        unsigned long long *tab = (unsigned long long *)ws_get(ctx, WS_TAB, sizeof(unsigned long long) * (size_t)std::max<int64_t>(tslots, 1));
        int32_t *tsize = (int32_t *)ws_get(ctx, WS_TSIZE, sizeof(int32_t) * nn);
        int32_t *tfail = (int32_t *)ws_get(ctx, WS_TFAIL, sizeof(int32_t) * nn);
        int32_t *tlist = (int32_t *)ws_get(ctx, WS_TLIST, sizeof(int32_t) * nn);
        if (!tab || !tsize || !tfail || !tlist) return JET_ENOMEM;
        JET_TRY(hipMemsetAsync(tfail, 0, sizeof(int32_t) * nn, s));
        a.toff = toff;
        a.tab = tab;
        a.tsize = tsize;
        a.tfail = tfail;
        a.tlist = tlist;
    }
    a.it = 0;
    k_ctl_setup<<<G, BLOCK, 0, s>>>(a);
    JET_TRY(hipGetLastError());
    // no wait here: the staging area of the upload is next written by the
    // final state read-back, ordered after it on the same stream
    pl.G = G;
    plan_roles(ctx, a, tot, pl);
    if (pl.table) {
        launch_tab_build(pl, s, 1);
        JET_TRY(hipGetLastError());
    }
    pl.grid_v = grid_v;
    pl.blkcnt = blkcnt;
    pl.lcnt = lcnt;
    pl.bins = bins;
    return JET_OK;
}

// Batch compaction: rebuilds the class lists (and the long-row chunk list)
// from the vertices of graphs still running, then re-plans the roles. Called
// between chunks of iterations, when nothing is in flight on the stream.
static int compact_lists(jet_context *ctx, Plan &pl, hipStream_t s)
{
    KArgs a = pl.plain;
    const int gv = pl.grid_v;
    const int32_t *ctot = pl.blkcnt + (size_t)gv * NCLS;
    k_bin_count_active<<<gv, BLOCK, 0, s>>>(a, pl.blkcnt);
    k_bin_scan<<<1, BLOCK, 0, s>>>(pl.blkcnt, gv);
    k_fill_bins_active<<<gv, BLOCK, 0, s>>>(a, pl.blkcnt, pl.bins);
    int32_t *lmeta = a.cnt + CNT_N;
    if (a.nlch > 0) {
        k_lchunk_count<<<gv, BLOCK, 0, s>>>(a.xadj, pl.bins, ctot, pl.lcnt);
        k_lchunk_scan<<<1, BLOCK, 0, s>>>(ctot, pl.lcnt, lmeta);
    }
    JET_TRY(hipGetLastError());
    int32_t *pin = (int32_t *)pinned_get(ctx, 4096);
    JET_TRY(hipMemcpyAsync(pin + 16, ctot, sizeof(int32_t) * NCLS, hipMemcpyDeviceToHost, s));
    if (a.nlch > 0) JET_TRY(hipMemcpyAsync(pin + 24, lmeta, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    JET_TRY(stream_wait(ctx, s));
    int32_t tot[NCLS];
    a.binoff[0] = 0;
    for (int c = 0; c < NCLS; c++) {
        tot[c] = pin[16 + c];
        a.binoff[c + 1] = a.binoff[c] + tot[c];
    }
    if (a.nlch > 0) {
        // never more chunks than at set-up, so the list and rows keep their room
        a.nlch = pin[24];
        if (a.nlch > 0) k_lchunk_fill<<<gv, BLOCK, 0, s>>>(ctot, pl.lcnt, (int2 *)a.lch);
        else a.lch = nullptr;
        JET_TRY(hipGetLastError());
    }
    const int grid_v = pl.grid_v;
    int32_t *blkcnt = pl.blkcnt, *lcnt = pl.lcnt, *bins = pl.bins;
    plan_roles(ctx, a, tot, pl);
    pl.grid_v = grid_v;
    pl.blkcnt = blkcnt;
    pl.lcnt = lcnt;
    pl.bins = bins;
    return JET_OK;
}

// Iterates until every graph is done: chunks of iterations, one sync each.
// Two consecutive iterations (launch indices of both parities) captured once
// as a HIP graph: kernels read only the parity of the launch index, so one
// pair replays any number of times. Replaying costs the host far less than
// enqueuing the ~15 kernels of every iteration one by one. The capture holds
// kernel launches only (no memset or copy nodes).
struct IterGraph {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    void reset()
    {
        if (x) (void)hipGraphExecDestroy(x);
        if (g) (void)hipGraphDestroy(g);
        x = nullptr;
        g = nullptr;
    }
    ~IterGraph() { reset(); }
};

static int capture_pair(jet_context *ctx, Plan &pl, IterGraph &ig)
{
    JET_TRY(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < 2; i++) {
        set_it(pl, i);
        launch_iteration(pl, ctx->cap);
    }
    const hipError_t e = hipStreamEndCapture(ctx->cap, &ig.g);
    if (e != hipSuccess) {
        ig.g = nullptr;
        return hip_status(ctx, e);
    }
    JET_TRY(hipGraphInstantiate(&ig.x, ig.g, nullptr, nullptr, 0));
    return JET_OK;
}

// Iterations launched between two looks at the loop state. One graph: the
// loop cannot end before the stall counter reaches
// stall_limit, so each chunk is what the counter still allows (at least 4,
// rounded up to whole pairs, at most 64 and never past max_iters), the
// first stall_limit + 1: few iterations run past the end and few waits are
// spent. A batch starts at 8 (4 without graph replay) and doubles up to 32.
static int single_chunk(const Ctl &c0, int left)
{
    if (c0.max_iters > 0) left = std::min(left, c0.max_iters - c0.t);
    return (std::min(std::max(left, 4), 64) + 1) & ~1;
}

static int next_chunk(bool single, const Ctl &c0, int chunk)
{
    if (single) return single_chunk(c0, c0.stall_limit - c0.stall);
    return std::min(chunk * 2, 32);
}

static int run_loop(jet_context *ctx, Plan &pl, bool prof, hipStream_t s, int &launched, const Ctl *single_ctl,
                    int async_iters = 0)
{
    if (async_iters > 0) {
        // JET_F_ASYNC: every iteration up to the cap is enqueued without a
        // look at the loop state; the controller ends the loop on the device
        // and later launches exit at once
        for (int i = 0; i < async_iters; i++) {
            set_it(pl, i);
            launch_iteration(pl, s);
        }
        launched = async_iters;
        JET_TRY(hipGetLastError());
        return JET_OK;
    }
    static_assert(64 + sizeof(Ctl) <= 4096, "pinned scratch holds the done count and one controller");
    int32_t *pin = (int32_t *)pinned_get(ctx, 4096);
    if (!pin) return JET_ENOMEM;
    Ctl *pin_ctl = (Ctl *)((char *)pin + 64);
    const bool single = single_ctl != nullptr;
    launched = 0;
    // a batch drops the vertices of finished graphs from its lists whenever
    // the number of running graphs has halved since the last rebuild
    int running_at_build = pl.G;
    auto maybe_compact = [&](int done, bool &rebuilt) -> int {
        rebuilt = false;
        const int running = pl.G - done;
        if (pl.G == 1 || running <= 0 || 2 * running > running_at_build) return JET_OK;
        running_at_build = running;
        rebuilt = true;
        return compact_lists(ctx, pl, s);
    };
    // loop state after a chunk: graphs done (and graph 0's controller)
    auto look = [&]() -> int {
        JET_TRY(hipMemcpyAsync(pin, pl.plain.cnt + CNT_DONE, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        if (single) JET_TRY(hipMemcpyAsync(pin_ctl, pl.plain.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        JET_TRY(stream_wait(ctx, s));
        return JET_OK;
    };
    const bool graphs = !prof && ctx->graphs && ctx->cap;
    int chunk = single ? single_chunk(*single_ctl, single_ctl->stall_limit + 1) : (graphs ? 8 : 4);
    if (graphs) {
        IterGraph ig;
        int st = capture_pair(ctx, pl, ig);
        if (st) return st;
        for (;;) {
            for (int i = 0; i < chunk; i += 2) JET_TRY(hipGraphLaunch(ig.x, s));
            launched += chunk;
            st = look();
            if (st) return st;
            if (pin[0] >= pl.G) break;
            bool rebuilt = false;
            st = maybe_compact(pin[0], rebuilt);
            if (st) return st;
            if (rebuilt) {
                ig.reset();
                st = capture_pair(ctx, pl, ig);
                if (st) return st;
            }
            chunk = next_chunk(single, *pin_ctl, chunk);
        }
        return JET_OK;
    }
    for (;;) {
        for (int i = 0; i < chunk; i++) {
            hipEvent_t ea = nullptr, eb = nullptr;
            if (prof && launched < KIND_LOG) {
                while ((int)ctx->prof_ev.size() < 2 * (launched + 1)) {
                    hipEvent_t e;
                    JET_TRY(hipEventCreate(&e));
                    ctx->prof_ev.push_back(e);
                }
                ea = ctx->prof_ev[2 * launched];
                eb = ctx->prof_ev[2 * launched + 1];
            }
            set_it(pl, launched);
            launch_iteration(pl, s, ea, eb);
            launched++;
        }
        JET_TRY(hipGetLastError());
        const int st = look();
        if (st) return st;
        if (pin[0] >= pl.G) break;
        bool rebuilt = false;
        const int st2 = maybe_compact(pin[0], rebuilt);
        if (st2) return st2;
        chunk = next_chunk(single, *pin_ctl, chunk);
    }
    return JET_OK;
}

// Final controller states: the read-back is enqueued here and lands in
// L.hc at take_state, after the caller's one synchronisation.
static int read_state(jet_context *ctx, Launch &L, const Plan &pl, hipStream_t s)
{
    Ctl *hcs = (Ctl *)((char *)pinned_get(ctx, 4096 + sizeof(Ctl) * (size_t)L.G) + 4096);
    JET_TRY(hipMemcpyAsync(hcs, pl.plain.ctl, sizeof(Ctl) * L.G, hipMemcpyDeviceToHost, s));
    return JET_OK;
}

static void take_state(jet_context *ctx, Launch &L)
{
    const Ctl *hcs = (const Ctl *)((const char *)ctx->pinned + 4096);
    memcpy(L.hc.data(), hcs, sizeof(Ctl) * L.G);
}

static void fill_stats(jet_stats *st, const Ctl &c, bool ret_iter)
{
    memset(st, 0, sizeof(*st));
    st->cut = ret_iter ? c.cut : c.cut_best;
    st->max_part_weight = ret_iter ? c.maxw : c.maxw_best;
    st->o = c.o;
    st->sigma = c.sigma;
    st->total_weight = c.W;
    st->balanced = st->max_part_weight <= c.o;
    st->iters = c.t;
    st->lp_iters = c.n_lp;
    st->rw_iters = c.n_rw;
    st->rs_iters = c.n_rs;
    st->levels = 1;
}

// One graph with k = 1 or n = 0: every vertex in part 0, nothing to refine.
static int refine_trivial(jet_context *ctx, const jet_csr *g, const jet_params *prm, int32_t *part,
                          int64_t *part_weights_out, jet_stats *stats, hipStream_t s)
{
    const int n = g->n, k = prm->k;
    if (n > 0) JET_TRY(hipMemsetAsync(part, 0, sizeof(int32_t) * n, s));
    int64_t W = n;
    if (n > 0 && g->vwgt) {
        std::vector<int32_t> vw(n);
        JET_TRY(hipMemcpyAsync(vw.data(), g->vwgt, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
        JET_TRY(stream_wait(ctx, s));
        W = 0;
        for (int32_t x : vw) W += x;
    }
    if (part_weights_out) {
        std::vector<int64_t> pw(k, 0);
        pw[0] = W;
        JET_TRY(hipMemcpyAsync(part_weights_out, pw.data(), sizeof(int64_t) * k, hipMemcpyHostToDevice, s));
    }
    JET_TRY(stream_wait(ctx, s));
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        stats->max_part_weight = W;
        stats->o = balance_limit(W, k, prm->lambda_ppm);
        stats->sigma = stats->o;
        stats->total_weight = W;
        stats->balanced = W <= stats->o;
        stats->levels = 1;
    }
    return JET_OK;
}

// Launch description of one graph refined on its own.
static void single_launch(Launch &L, const jet_csr *g, const jet_params *prm, int32_t *part,
                          jet_trace_rec *trace_dev, int32_t trace_cap)
{
    L.G = 1;
    L.u = *g;
    L.part_in = part;
    L.best = part;
    L.ktot = prm->k;
    L.kmax = prm->k;
    L.ntile = std::max(1, div_up(g->n, TILE));
    L.tsum_cap = (int64_t)L.ntile * prm->k;
    L.trace_dev = trace_dev;
    L.hc.assign(1, make_ctl(prm, g->n));
    Ctl &c = L.hc[0];
    c.t0 = 0;
    c.ntiles = L.ntile;
    c.rowbase = 0;
    c.trace_off = 0;
    c.trace_cap = trace_dev ? trace_cap : 0;
}

// Results of a JET_F_ASYNC refinement, filled in by a host function the
// stream runs after the call's last copy (no HIP call inside).
struct AsyncDone {
    const Ctl *ctl;                     // final controller state (pinned staging)
    const jet_trace_rec *trace_stage;   // trace records (pinned staging)
    jet_stats *stats;
    jet_trace_rec *trace_host;
    int32_t trace_cap;
    int32_t *trace_count, *trace_total;
    bool ret_iter;
};

static void async_done(void *p)
{
    AsyncDone *d = (AsyncDone *)p;
    const Ctl &c = *d->ctl;
    if (d->stats) fill_stats(d->stats, c, d->ret_iter);
    const int ntr = std::min(c.t, c.trace_cap);
    if (d->trace_host && ntr > 0) memcpy(d->trace_host, d->trace_stage, sizeof(jet_trace_rec) * (size_t)ntr);
    if (d->trace_count) *d->trace_count = ntr;
    if (d->trace_total) *d->trace_total = c.t;
    delete d;
}

int refine_level(jet_context *ctx, const jet_csr *g, const jet_params *prm, int32_t *part,
                 int64_t *part_weights_out, jet_stats *stats, jet_trace_rec *trace_host, int32_t trace_cap,
                 int32_t *trace_count, int32_t *trace_total, hipStream_t s, int64_t cut0)
{
    int st = check_params(g, prm);
    if (st) return st;
    const int n = g->n, k = prm->k;
    const bool async = prm->flags & JET_F_ASYNC;
    if (async && (prm->max_iters <= 0 || (prm->flags & JET_F_PROFILE))) return JET_EINVAL;
    if (trace_count) *trace_count = 0;
    if (trace_total) *trace_total = 0;
    if (k == 1 || n == 0) return refine_trivial(ctx, g, prm, part, part_weights_out, stats, s);
    // the staging of an asynchronous call's results is sized before any
    // copy into it is enqueued (growing it later would free it under them)
    const size_t stage_off = (4096 + sizeof(Ctl) + 63) & ~(size_t)63;
    if (async && !pinned_get(ctx, stage_off + sizeof(jet_trace_rec) * (size_t)std::max(trace_cap, 0)))
        return JET_ENOMEM;
    if (prm->flags & JET_F_VALIDATE) {
        st = validate_full_csr(ctx, g, s);
        if (st) return st;
    }
    JET_TRY(hipEventRecord(ctx->ev[0], s));
    jet_trace_rec *trace_dev = nullptr;
    if (trace_host && trace_cap > 0) {
        trace_dev = (jet_trace_rec *)ws_get(ctx, WS_TRACE, sizeof(jet_trace_rec) * (size_t)trace_cap);
        if (!trace_dev) return JET_ENOMEM;
    }
    Launch L;
    single_launch(L, g, prm, part, trace_dev, trace_cap);
    L.cut0 = cut0;
    Plan pl;
    st = setup(ctx, L, pl, s, nullptr);
    if (st) return st;
    JET_TRY(hipEventRecord(ctx->ev[1], s));
    const bool prof = prm->flags & JET_F_PROFILE;
    int launched = 0;
    st = run_loop(ctx, pl, prof, s, launched, &L.hc[0], async ? prm->max_iters : 0);
    if (st) return st;
    k_copy_best<<<pl.grid_flat, BLOCK, 0, s>>>(pl.plain);
    JET_TRY(hipEventRecord(ctx->ev[2], s));
    if (prm->flags & JET_F_RETURN_ITER)
        k_copy_iter<<<pl.grid_flat, BLOCK, 0, s>>>(pl.plain, part);
    if (part_weights_out)
        JET_TRY(hipMemcpyAsync(part_weights_out, (prm->flags & JET_F_RETURN_ITER) ? pl.plain.w : pl.plain.wbest,
                               sizeof(int64_t) * k, hipMemcpyDeviceToDevice, s));
    st = read_state(ctx, L, pl, s);
    if (st) return st;
    if (async) {
        // results land in pinned staging; a host function on the stream hands
        // them to the caller once everything before it has run
        char *pin = (char *)ctx->pinned;
        jet_trace_rec *stage = (jet_trace_rec *)(pin + stage_off);
        const int ncopy = std::min(launched, L.hc[0].trace_cap);
        if (trace_dev && ncopy > 0)
            JET_TRY(hipMemcpyAsync(stage, trace_dev, sizeof(jet_trace_rec) * ncopy, hipMemcpyDeviceToHost, s));
        AsyncDone *d = new (std::nothrow) AsyncDone{(const Ctl *)(pin + 4096), stage, stats, trace_host, trace_cap,
                                                    trace_count, trace_total, (prm->flags & JET_F_RETURN_ITER) != 0};
        if (!d) return JET_ENOMEM;
        const hipError_t e = hipLaunchHostFunc(s, async_done, d);
        if (e != hipSuccess) {
            delete d;
            return hip_status(ctx, e);
        }
        return JET_OK;
    }
    // records exist for the iterations run, at most one per launched iteration
    const int ncopy = std::min(launched, L.hc[0].trace_cap);
    if (trace_dev && ncopy > 0)
        JET_TRY(hipMemcpyAsync(trace_host, trace_dev, sizeof(jet_trace_rec) * ncopy, hipMemcpyDeviceToHost, s));
    JET_TRY(hipEventRecord(ctx->ev[3], s));
    JET_TRY(stream_wait(ctx, s));
    take_state(ctx, L);
    const Ctl &hc = L.hc[0];
    const int ntr = std::min(hc.t, hc.trace_cap);
    if (trace_count) *trace_count = ntr;
    if (trace_total) *trace_total = hc.t;
    float ms_gain = 0.f;
    int gain_passes = 0;
    if (prof) {
        const int nk = std::min(hc.t, KIND_LOG);
        std::vector<int8_t> kinds(std::max(nk, 1));
        if (nk > 0) {
            JET_TRY(hipMemcpyAsync(kinds.data(), pl.plain.kinds, nk, hipMemcpyDeviceToHost, s));
            JET_TRY(stream_wait(ctx, s));
        }
        // launch i ran iteration i (the kind log is written before t advances)
        for (int i = 0; i < nk; i++) {
            if (kinds[i] != KIND_LP) continue;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ctx->prof_ev[2 * i], ctx->prof_ev[2 * i + 1]) == hipSuccess) {
                ms_gain += ms;
                gain_passes++;
            }
        }
    }
    if (stats) {
        fill_stats(stats, hc, prm->flags & JET_F_RETURN_ITER);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[3]);
        stats->ms_total = ms;
        (void)hipEventElapsedTime(&ms, ctx->ev[1], ctx->ev[2]);
        stats->ms_refine = ms;
        (void)hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]);
        stats->ms_init = ms;
        if (prof) {
            stats->ms_gain = ms_gain;
            stats->gain_passes = gain_passes;
            stats->gain_entries = hc.prof_e;
            stats->gain_rows = hc.prof_r;
            stats->gain_vertices = hc.prof_v;
        }
    }
    return JET_OK;
}

// Autotuner of a batch's launch sequence: picks how waves walk the class
// lists (static stretches, or work-queue tiles of 16 or 64 visits of their
// role) and, where k allows both, 4- or 8-lane groups for the small rows, by
// timing one dry gain pass of each choice over the batch itself
// (k_tune_prep). Every choice gives the same results; only the time
// differs. The choice is recorded in the context per batch shape (graph
// count, size and CSR-entry scales, largest k), so repeated calls on batches
// of that shape reuse it; small batches take static walks.
// JET_BATCH_TILE (0 = static) / JET_BATCH_GROUP force a choice.
static uint64_t batch_signature(const Plan &pl, int64_t nnz)
{
    auto lg = [](int64_t x) { return (uint64_t)(64 - __builtin_clzll((unsigned long long)(x | 1))); };
    return ((uint64_t)pl.G << 32) ^ (lg(pl.tab.n) << 24) ^ (lg(nnz) << 16) ^ (uint64_t)pl.tab.k;
}

static int tune_batch(jet_context *ctx, Plan &pl, int64_t nnz, hipStream_t s)
{
    const char *et = getenv("JET_BATCH_TILE"), *eg = getenv("JET_BATCH_GROUP");
    int tile = 0;
    bool g8 = pl.tab.k > K_G4;
    const uint64_t sig = batch_signature(pl, nnz);
    bool cached = false;
    for (const auto &e : ctx->tune_cache)
        if (e.first == sig) {
            tile = e.second & 0xFFFF;
            g8 = (e.second >> 16) != 0;
            cached = true;
        }
    if (et || eg || (!cached && nnz < ((int64_t)1 << 20))) {
        if (et && atoi(et) >= 0) tile = atoi(et);
        if (eg) g8 = atoi(eg) == 8 || pl.tab.k > K_G4;
    } else if (!cached) {
        const int G = pl.G, n = pl.tab.n;
        Ctl *ctl2 = (Ctl *)ws_get(ctx, WS_TUNE_CTL, sizeof(Ctl) * (size_t)G);
        int32_t *cnt2 = (int32_t *)ws_get(ctx, WS_TUNE_CNT, sizeof(int32_t) * (CNT_N + 2 + 2 * NQC));
        int2 *rec2 = (int2 *)ws_get(ctx, WS_TUNE_REC, sizeof(int2) * (size_t)std::max(n, 1));
        int64_t *st2 = (int64_t *)ws_get(ctx, WS_TUNE_STAT, sizeof(int64_t) * NSTAT * NSHARD * (size_t)G);
        if (!ctl2 || !cnt2 || !rec2 || !st2) return JET_ENOMEM;
        int32_t *wq2 = cnt2 + CNT_N + 2;
        k_tune_prep<<<G, BLOCK, 0, s>>>(pl.plain, ctl2, cnt2);
        constexpr int NT = 3;
        const int tiles[NT] = {0, 16, 64};
        const int ng = pl.tab.k <= K_G4 ? 2 : 1;
        hipEvent_t ev[2 * NT * 2];
        int ne = 0;
        hipError_t e = hipSuccess;
        for (int i = 0; i < 2 * NT * ng; i++) {
            e = hipEventCreate(&ev[i]);
            if (e != hipSuccess) break;
            ne++;
        }
        if (e != hipSuccess) {
            for (int i = 0; i < ne; i++) (void)hipEventDestroy(ev[i]);
            return hip_status(ctx, e);
        }
        int c = 0;
        for (int gi = 0; gi < ng; gi++)
            for (int ti = 0; ti < NT; ti++, c++) {
                Plan dp = pl;
                for (KArgs *k : {&dp.tab, &dp.plain}) {
                    k->ctl = ctl2;
                    k->cnt = cnt2;
                    k->rec = rec2;
                    k->bstat = st2;
                    k->wq = wq2;
                    k->wtile = tiles[ti];
                    k->it = 0;
                }
                dp.small_g8 = gi == 1;
                JET_TRY(hipMemsetAsync(st2, 0, sizeof(int64_t) * NSTAT * NSHARD * (size_t)G, s));
                JET_TRY(hipMemsetAsync(wq2, 0, sizeof(int32_t) * 2 * NQC, s));
                JET_TRY(hipEventRecord(ev[2 * c], s));
                launch_gain_t<true>(dp, s);
                JET_TRY(hipEventRecord(ev[2 * c + 1], s));
            }
        JET_TRY(hipGetLastError());
        JET_TRY(stream_wait(ctx, s));
        float best = 1e30f;
        c = 0;
        for (int gi = 0; gi < ng; gi++)
            for (int ti = 0; ti < NT; ti++, c++) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, ev[2 * c], ev[2 * c + 1]) == hipSuccess && ms < best) {
                    best = ms;
                    tile = tiles[ti];
                    g8 = gi == 1 || pl.tab.k > K_G4;
                }
            }
        for (int i = 0; i < ne; i++) (void)hipEventDestroy(ev[i]);
        ctx->tune_cache.emplace_back(sig, tile | ((g8 ? 1 : 0) << 16));
    }
    pl.tab.wtile = pl.plain.wtile = tile;
    pl.small_g8 = g8 && pl.tab.k <= K_G4;
    return JET_OK;
}

int refine_batch(jet_context *ctx, int count, const jet_csr *graphs, const jet_params *params, int32_t *const *parts,
                 jet_stats *stats, jet_trace *traces, hipStream_t s)
{
    if (count < 0 || (count > 0 && (!graphs || !params || !parts))) return JET_EINVAL;
    for (int i = 0; i < count; i++) {
        const int st = check_params(&graphs[i], &params[i]);
        if (st) return st;
        if (graphs[i].n > 0 && !parts[i]) return JET_EINVAL;
        if (traces && traces[i].cap > 0 && !traces[i].recs) return JET_EINVAL;
        if (params[i].flags & JET_F_ASYNC) return JET_EINVAL;
    }
    for (int i = 0; i < count; i++)
        if (params[i].flags & JET_F_VALIDATE) {
            const int st = validate_full_csr(ctx, &graphs[i], s);
            if (st) return st;
        }
    // graphs with one part or no vertex need no refinement
    std::vector<int> act;
    for (int i = 0; i < count; i++) {
        if (traces) {
            traces[i].count = 0;
            traces[i].total = 0;
        }
        if (params[i].k == 1 || graphs[i].n == 0) {
            const int st = refine_trivial(ctx, &graphs[i], &params[i], parts[i], nullptr, stats ? &stats[i] : nullptr, s);
            if (st) return st;
        } else {
            act.push_back(i);
        }
    }
    const int G = (int)act.size();
    if (G == 0) return JET_OK;
    JET_TRY(hipEventRecord(ctx->ev[0], s));
    // union layout
    Launch L;
    L.G = G;
    L.hc.resize(G);
    std::vector<UDesc> hd(G);
    int64_t N = 0, NNZ = 0, tsum = 0, trace_total = 0;
    int64_t ktot = 0, ntile = 0;
    int kmax = 0;
    bool any_vw = false, any_ew = false;
    for (int j = 0; j < G; j++) {
        const int i = act[j];
        const jet_csr &g = graphs[i];
        const jet_params &p = params[i];
        Ctl c = make_ctl(&p, g.n);
        c.voff = (int32_t)N;
        c.poff = (int32_t)ktot;
        c.t0 = (int32_t)ntile;
        c.ntiles = div_up(g.n, TILE);
        c.rowbase = tsum;
        c.trace_off = (int32_t)trace_total;
        c.trace_cap = traces ? std::max(traces[i].cap, 0) : 0;
        L.hc[j] = c;
        UDesc &d = hd[j];
        d.xadj = g.xadj;
        d.adj = g.adjncy;
        d.vw = g.vwgt;
        d.ew = g.adjwgt;
        d.part = parts[i];
        d.eoff = NNZ;
        d.nnz = g.nnz;
        d.voff = (int32_t)N;
        d.n = g.n;
        d.ret_iter = (p.flags & JET_F_RETURN_ITER) ? 1 : 0;
        d.pad = 0;
        N += g.n;
        NNZ += g.nnz;
        ktot += p.k;
        ntile += c.ntiles;
        tsum += (int64_t)c.ntiles * p.k;
        trace_total += c.trace_cap;
        kmax = std::max(kmax, p.k);
        any_vw = any_vw || g.vwgt;
        any_ew = any_ew || g.adjwgt;
        if (N >= INT32_MAX || ktot >= INT32_MAX || ntile >= INT32_MAX || trace_total >= INT32_MAX) return JET_ELIMIT;
    }
    L.ktot = (int)ktot;
    L.kmax = kmax;
    L.ntile = (int)ntile;
    L.tsum_cap = tsum;
    std::vector<int32_t> maps(ntile + ktot);  // graph of each tile, then of each global part
    for (int j = 0; j < G; j++) {
        for (int t = 0; t < L.hc[j].ntiles; t++) maps[L.hc[j].t0 + t] = j;
        for (int p = 0; p < L.hc[j].k; p++) maps[ntile + L.hc[j].poff + p] = j;
    }
    int64_t *uxadj = (int64_t *)ws_get(ctx, WS_U_XADJ, sizeof(int64_t) * (size_t)(N + 1));
    int32_t *uadj = (int32_t *)ws_get(ctx, WS_U_ADJ, sizeof(int32_t) * (size_t)std::max<int64_t>(NNZ, 1));
    int32_t *uvw = any_vw ? (int32_t *)ws_get(ctx, WS_U_VW, sizeof(int32_t) * (size_t)N) : nullptr;
    int32_t *uew = any_ew ? (int32_t *)ws_get(ctx, WS_U_EW, sizeof(int32_t) * (size_t)std::max<int64_t>(NNZ, 1)) : nullptr;
    int32_t *uvg = (int32_t *)ws_get(ctx, WS_U_VG, sizeof(int32_t) * (size_t)N);
    int32_t *up0 = (int32_t *)ws_get(ctx, WS_U_P0, sizeof(int32_t) * (size_t)N);
    int32_t *ubest = (int32_t *)ws_get(ctx, WS_U_BEST, sizeof(int32_t) * (size_t)N);
    UDesc *udesc = (UDesc *)ws_get(ctx, WS_U_DESC, sizeof(UDesc) * (size_t)G + 64);
    int32_t *umaps = (int32_t *)ws_get(ctx, WS_TG, sizeof(int32_t) * (size_t)(ntile + ktot));
    jet_trace_rec *trace_dev = nullptr;
    if (trace_total > 0) trace_dev = (jet_trace_rec *)ws_get(ctx, WS_TRACE, sizeof(jet_trace_rec) * (size_t)trace_total);
    if (!uxadj || !uadj || (any_vw && !uvw) || (any_ew && !uew) || !uvg || !up0 || !ubest || !udesc || !umaps ||
        (trace_total > 0 && !trace_dev))
        return JET_ENOMEM;
    int32_t *ubad = (int32_t *)((char *)udesc + sizeof(UDesc) * (size_t)G);
    JET_TRY(hipMemcpyAsync(udesc, hd.data(), sizeof(UDesc) * G, hipMemcpyHostToDevice, s));
    JET_TRY(hipMemcpyAsync(umaps, maps.data(), sizeof(int32_t) * maps.size(), hipMemcpyHostToDevice, s));
    JET_TRY(hipMemsetAsync(ubad, 0, sizeof(int32_t), s));
    const int grid_v = std::max(1, std::min(div_up(N, BLOCK), ctx->num_cu * 8));
    const int grid_e = std::max(1, std::min(div_up(NNZ, BLOCK), ctx->num_cu * 16));
    k_union_vertices<<<grid_v, BLOCK, 0, s>>>(udesc, G, (int)N, NNZ, uxadj, uvw, uvg, up0, ubad);
    if (NNZ > 0) k_union_edges<<<grid_e, BLOCK, 0, s>>>(udesc, G, NNZ, uadj, uew, ubad);
    JET_TRY(hipGetLastError());
    int32_t *hbad = (int32_t *)pinned_get(ctx, 4096);
    if (!hbad) return JET_ENOMEM;
    JET_TRY(hipMemcpyAsync(hbad, ubad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    JET_TRY(stream_wait(ctx, s));
    if (hbad[0]) return JET_EGRAPH;
    L.u.n = (int32_t)N;
    L.u.nnz = NNZ;
    L.u.xadj = uxadj;
    L.u.adjncy = uadj;
    L.u.vwgt = uvw;
    L.u.adjwgt = uew;
    L.vg = uvg;
    L.tg = umaps;
    L.pg = umaps + ntile;
    L.part_in = up0;
    L.best = ubest;
    L.trace_dev = trace_dev;
    Plan pl;
    int st = setup(ctx, L, pl, s, nullptr);
    if (st) return st;
    st = tune_batch(ctx, pl, NNZ, s);
    if (st) return st;
    JET_TRY(hipEventRecord(ctx->ev[1], s));
    int launched = 0;
    st = run_loop(ctx, pl, false, s, launched, nullptr);
    if (st) return st;
    k_copy_best<<<pl.grid_flat, BLOCK, 0, s>>>(pl.plain);
    JET_TRY(hipEventRecord(ctx->ev[2], s));
    k_union_scatter<<<grid_v, BLOCK, 0, s>>>(udesc, G, (int)N, pl.plain.P, ubest);
    JET_TRY(hipGetLastError());
    st = read_state(ctx, L, pl, s);
    if (st) return st;
    if (traces)
        for (int j = 0; j < G; j++) {
            const Ctl &c = L.hc[j];  // configuration: trace offset and capacity
            const int ncopy = std::min(launched, c.trace_cap);
            if (ncopy > 0)
                JET_TRY(hipMemcpyAsync(traces[act[j]].recs, trace_dev + c.trace_off, sizeof(jet_trace_rec) * ncopy,
                                       hipMemcpyDeviceToHost, s));
        }
    JET_TRY(hipEventRecord(ctx->ev[3], s));
    JET_TRY(stream_wait(ctx, s));
    take_state(ctx, L);
    if (traces)
        for (int j = 0; j < G; j++) {
            jet_trace &tr = traces[act[j]];
            const Ctl &c = L.hc[j];
            tr.count = std::min(c.t, c.trace_cap);
            tr.total = c.t;
        }
    if (stats) {
        float ms_total = 0, ms_refine = 0, ms_init = 0;
        (void)hipEventElapsedTime(&ms_total, ctx->ev[0], ctx->ev[3]);
        (void)hipEventElapsedTime(&ms_refine, ctx->ev[1], ctx->ev[2]);
        (void)hipEventElapsedTime(&ms_init, ctx->ev[0], ctx->ev[1]);
        for (int j = 0; j < G; j++) {
            jet_stats &sj = stats[act[j]];
            fill_stats(&sj, L.hc[j], params[act[j]].flags & JET_F_RETURN_ITER);
            sj.ms_total = ms_total;
            sj.ms_refine = ms_refine;
            sj.ms_init = ms_init;
            sj.batch_tile = pl.tab.wtile;
            sj.batch_group = (pl.tab.k <= K_G4 && !pl.small_g8) ? 4 : 8;
        }
    }
    return JET_OK;
}

}  // namespace jet

using namespace jet;

// --------------------------------------------------------------- C ABI ------

// Workspace of jet_refine_noalloc: one static array per GPU, part of the code
// object. Host code never passes its name to a kernel (on the host the name
// is a stand-in, not a device address): jet_context_create looks up each
// device's address once, with that device current, and the call hands that
// address to ws_get.
static __device__ __align__(256) unsigned char scratch[JET_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of this device's scratch array (the device must be current).
int scratch_lookup(jet_context *ctx, int device, char **out)
{
    *out = nullptr;
    if (device < 0 || device >= MAX_DEVICES) return JET_ELIMIT;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_status(ctx, e != hipSuccess ? e : hipErrorInvalidSymbol);
        g_scratch_ptr[device] = (char *)ptr;
    }
    *out = g_scratch_ptr[device];
    return JET_OK;
}
}  // namespace

// The refinement loop reads its state back many times per partition; a
// thread that sleeps in the runtime until the stream drains wakes up tens of
// microseconds late each time, so the wait polls an event instead.
hipError_t jet::stream_wait(jet_context *ctx, hipStream_t s)
{
    if (!ctx->poll_wait || !ctx->wait_ev) return hipStreamSynchronize(s);
    hipError_t e = hipEventRecord(ctx->wait_ev, s);
    if (e != hipSuccess) return e;
    for (;;) {
        e = hipEventQuery(ctx->wait_ev);
        if (e != hipErrorNotReady) return e;
        __builtin_ia32_pause();
    }
}

extern "C" int jet_context_create(jet_context **out, int device)
{
    if (!out) return JET_EINVAL;
    *out = nullptr;
    jet_context *ctx = new (std::nothrow) jet_context();
    if (!ctx) return JET_ENOMEM;
    ctx->device = device;
    ctx->bufs.resize(WS_COUNT);
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) {
        int st = hip_status(ctx, e);
        delete ctx;
        return st;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        ctx->num_cu = prop.multiProcessorCount;
    // staging for one controller and the loop state: large enough that a
    // single-graph call never grows it (jet_refine_noalloc allocates nothing)
    if (!pinned_get(ctx, 16384)) {
        delete ctx;
        return JET_ENOMEM;
    }
    {
        const int st = scratch_lookup(ctx, device, &ctx->scratch);
        if (st) {
            jet_context_destroy(ctx);
            return st;
        }
    }
    const char *ng = getenv("JET_NO_GRAPH");
    ctx->graphs = !(ng && ng[0] == '1');
    const char *bw = getenv("JET_BLOCKING_WAIT");
    ctx->poll_wait = !(bw && bw[0] == '1');
    const char *p8 = getenv("JET_NO_PART8");
    ctx->part8 = !(p8 && p8[0] == '1');
    e = hipEventCreateWithFlags(&ctx->wait_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        int st = hip_status(ctx, e);
        jet_context_destroy(ctx);
        return st;
    }
    e = hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        int st = hip_status(ctx, e);
        jet_context_destroy(ctx);
        return st;
    }
    for (auto &ev : ctx->ev) {
        e = hipEventCreate(&ev);
        if (e != hipSuccess) {
            int st = hip_status(ctx, e);
            jet_context_destroy(ctx);
            return st;
        }
    }
    *out = ctx;
    return JET_OK;
}

extern "C" void jet_context_destroy(jet_context *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    for (auto &b : ctx->bufs)
        if (b.ptr) (void)hipFree(b.ptr);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    for (auto &ev : ctx->ev)
        if (ev) (void)hipEventDestroy(ev);
    for (auto ev : ctx->prof_ev) (void)hipEventDestroy(ev);
    if (ctx->wait_ev) (void)hipEventDestroy(ctx->wait_ev);
    ctx->part_arena.release();
    if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
    if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
    if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
    if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
    delete ctx;
}

extern "C" int jet_last_hip_error(const jet_context *ctx) { return ctx ? ctx->last_hip : 0; }

extern "C" const char *jet_strerror(int status)
{
    switch (status) {
    case JET_OK: return "ok";
    case JET_EINVAL: return "invalid parameter";
    case JET_EGRAPH: return "malformed CSR graph";
    case JET_EPART: return "part id out of range";
    case JET_EOVERFLOW: return "weight too large (total vertex weight or a weighted degree >= 2^31)";
    case JET_ENOMEM: return "out of memory";
    case JET_EHIP: return "HIP runtime error";
    case JET_EAGAIN: return "try again";
    case JET_ELIMIT: return "size limit exceeded";
    default: return "unknown status";
    }
}

extern "C" int jet_refine(jet_context *ctx, const jet_csr *g, const jet_params *params, int32_t *part,
                          int64_t *part_weights_out, jet_stats *stats, jet_trace *trace, void *stream)
{
    if (!ctx || !g || !params || (!part && g->n > 0)) return JET_EINVAL;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_status(ctx, e);
    // the trace counts are written by the call (or, with JET_F_ASYNC, by the
    // host function that completes it on the stream)
    return refine_level(ctx, g, params, part, part_weights_out, stats, trace ? trace->recs : nullptr,
                        trace ? trace->cap : 0, trace ? &trace->count : nullptr, trace ? &trace->total : nullptr,
                        (hipStream_t)stream);
}

// Upper bound of the workspace jet_refine carves for one graph (each slot
// rounded up to the 256-byte alignment of the bump allocation). Long rows
// (> 1024 entries) number at most nnz / 1025, their chunks at most
// nnz / 1024 + their count.
static size_t noalloc_need(int64_t n, int64_t nnz, int64_t k, int64_t trace_cap, int num_cu)
{
    auto al = [](size_t b) { return (std::max(b, (size_t)16) + 255) & ~(size_t)255; };
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    const int64_t ntile = std::max<int64_t>(1, (n + TILE - 1) / TILE);
    const int64_t grid_v = std::max<int64_t>(1, std::min<int64_t>((n + BLOCK - 1) / BLOCK, (int64_t)num_cu * 4));
    const int64_t nL = nnz / (M_MAXDEG + 1), nch = nnz / LCHUNK + nL;  // bounds
    size_t b = 0;
    if (trace_cap > 0) b += al(sizeof(jet_trace_rec) * (size_t)trace_cap);
    b += al(nn * 2) + al(nn * 8) + al(nn * 4) + al(nn * 4) + al(nn) + al(nn * 4) + al(nn) + al(nn * 4);
    b += al(nn) + al(nn * 4) + al(nn * 4) + al(nn * 4);  // byte parts, packed (old, new) parts, records and F, at their largest
    b += al(4 * (size_t)(nnz / 4096 + 1));   // row marks of the edge pass
    b += al(sizeof(int64_t) * NSTAT * NSHARD) + al(sizeof(int32_t) * (CNT_N + 2)) + al(sizeof(Ctl));
    b += al(sizeof(int64_t) * (4 * (size_t)k + 9)) + al(sizeof(int32_t) * (3 * (size_t)k + 8)) + al(2 * (size_t)k + 16);
    b += al(sizeof(int64_t) * (size_t)k * NSLOT) + al(sizeof(int32_t) * (size_t)(ntile * k)) + al(8 * (size_t)ntile);
    b += al(KIND_LOG) + al(sizeof(int32_t) * (size_t)(grid_v + 1) * NCLS) + al(4 * (nn + 1)) + al(16);
    if (nL > 0) b += al(8 * (size_t)nch) + al(4 * std::min((size_t)nch * (size_t)k, (size_t)128 << 20)) +
                     al(8 * (size_t)nL);
    return b;
}

extern "C" int jet_refine_noalloc(jet_context *ctx, const jet_csr *g, const jet_params *params, int32_t *part,
                                  int64_t *part_weights_out, jet_stats *stats, jet_trace *trace, void *stream)
{
    if (!ctx || !g || !params || (!part && g->n > 0)) return JET_EINVAL;
    int st = check_params(g, params);
    if (st) return st;
    if (params->k < 2 || (params->flags & (JET_F_VALIDATE | JET_F_PROFILE | JET_F_ASYNC | JET_F_CONN_TABLE)))
        return JET_EINVAL;
    if (!ctx->scratch) return JET_EHIP;
    const int32_t tcap = trace && trace->recs ? std::max(trace->cap, 0) : 0;
    if (noalloc_need(g->n, g->nnz, params->k, tcap, ctx->num_cu) > (size_t)JET_NOALLOC_SCRATCH_BYTES)
        return JET_ELIMIT;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_status(ctx, e);
    hipStream_t s = (hipStream_t)stream;
    if (trace) {
        trace->count = 0;
        trace->total = 0;
    }
    if (g->n == 0) {
        // nothing to refine: every part is empty
        if (part_weights_out) JET_TRY(hipMemsetAsync(part_weights_out, 0, sizeof(int64_t) * params->k, s));
        JET_TRY(stream_wait(ctx, s));
        if (stats) {
            memset(stats, 0, sizeof(*stats));
            stats->balanced = 1;
            stats->levels = 1;
        }
        return JET_OK;
    }
    // every workspace slot from the scratch array, iterations launched
    // directly (no graph instantiation); restored on every return path
    struct Mode {
        jet_context *c;
        bool graphs;
        Mode(jet_context *cc) : c(cc), graphs(cc->graphs)
        {
            c->scratch_on = true;
            c->scratch_off = 0;
            c->graphs = false;
        }
        ~Mode()
        {
            c->scratch_on = false;
            c->scratch_off = 0;
            c->graphs = graphs;
        }
    } mode(ctx);
    int32_t cnt = 0, tot = 0;
    st = refine_level(ctx, g, params, part, part_weights_out, stats, trace ? trace->recs : nullptr,
                      trace ? trace->cap : 0, &cnt, &tot, s);
    if (trace) {
        trace->count = cnt;
        trace->total = tot;
    }
    return st;
}

extern "C" int jet_gather_ceiling(jet_context *ctx, const jet_csr *g, const int32_t *part, int32_t k, int32_t reps,
                                  float *ms, void *stream)
{
    if (!ctx || !g || !part || !ms || reps < 1 || k < 1 || g->n < 1 || g->nnz < 1 || !g->xadj || !g->adjncy)
        return JET_EINVAL;
    if (k > KMAX) return JET_ELIMIT;
    hipStream_t s = (hipStream_t)stream;
    JET_TRY(hipSetDevice(ctx->device));
    // ids are checked against n (cheap O(nnz) pass) before any gather; the
    // weight limits guard arithmetic this pass does not do
    int st = check_graph(ctx, g, 0, s);
    if (st && st != JET_EOVERFLOW) return st;
    void *P = ws_get(ctx, WS_P, sizeof(uint16_t) * (size_t)g->n);
    unsigned long long *out = (unsigned long long *)ws_get(ctx, WS_WDEG, 16);
    if (!P || !out) return JET_ENOMEM;
    const int grid_v = std::max(1, std::min(div_up(g->n, BLOCK), ctx->num_cu * 4));
    const int grid = ctx->num_cu * 8;
    const bool bytes = k <= 256;
    auto pass = [&]() {
        if (bytes) k_gather_ceiling<uint8_t><<<grid, BLOCK, 0, s>>>(g->adjncy, g->adjwgt, (const uint8_t *)P, g->nnz, out);
        else k_gather_ceiling<uint16_t><<<grid, BLOCK, 0, s>>>(g->adjncy, g->adjwgt, (const uint16_t *)P, g->nnz, out);
    };
    if (bytes) k_part_narrow<uint8_t><<<grid_v, BLOCK, 0, s>>>(part, g->n, (uint8_t *)P);
    else k_part_narrow<uint16_t><<<grid_v, BLOCK, 0, s>>>(part, g->n, (uint16_t *)P);
    pass();  // warm-up
    JET_TRY(hipEventRecord(ctx->ev[0], s));
    for (int r = 0; r < reps; r++) pass();
    JET_TRY(hipEventRecord(ctx->ev[1], s));
    JET_TRY(hipGetLastError());
    JET_TRY(stream_wait(ctx, s));
    float t = 0.f;
    JET_TRY(hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[1]));
    *ms = t / reps;
    return JET_OK;
}

extern "C" int jet_refine_batch(jet_context *ctx, int32_t count, const jet_csr *graphs, const jet_params *params,
                                int32_t *const *parts, jet_stats *stats, jet_trace *traces, void *stream)
{
    if (!ctx) return JET_EINVAL;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_status(ctx, e);
    return refine_batch(ctx, count, graphs, params, parts, stats, traces, (hipStream_t)stream);
}

// Shared set-up of the single-step entry points: one graph, a private copy of
// the partition, the step outputs wired in.
static int step_setup(jet_context *ctx, const jet_csr *g, const jet_params *params, const int32_t *part,
                      const DebugOut &dbg, Launch &L, Plan &pl, hipStream_t s)
{
    const int n = g->n;
    int32_t *p0 = (int32_t *)ws_get(ctx, WS_H0, sizeof(int32_t) * n);
    if (!p0) return JET_ENOMEM;
    JET_TRY(hipMemcpyAsync(p0, part, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    if (params->flags & JET_F_VALIDATE) {
        const int st = validate_full_csr(ctx, g, s);
        if (st) return st;
    }
    single_launch(L, g, params, p0, nullptr, 0);
    return setup(ctx, L, pl, s, &dbg);
}

extern "C" int jet_lp_step(jet_context *ctx, const jet_csr *g, const jet_params *params, const int32_t *part,
                           const uint8_t *locked, int32_t *pd, int64_t *F, int64_t *conn_s, uint8_t *inX,
                           int64_t *F2, uint8_t *move, void *stream)
{
    if (!ctx || !g || !params) return JET_EINVAL;
    int st = check_params(g, params);
    if (st) return st;
    const int n = g->n;
    if (n > 0 && (!part || !locked || !pd || !F || !conn_s || !inX || !F2 || !move)) return JET_EINVAL;
    if (params->k < 2) return JET_EINVAL;
    if (n == 0) return JET_OK;
    hipStream_t s = (hipStream_t)stream;
    JET_TRY(hipSetDevice(ctx->device));
    DebugOut dbg;
    dbg.F = F;
    dbg.cs = conn_s;
    dbg.F2 = F2;
    dbg.pd = pd;
    Launch L;
    Plan pl;
    st = step_setup(ctx, g, params, part, dbg, L, pl, s);
    if (st) return st;
    set_it(pl, 0);
    k_step_defaults<<<pl.grid_flat, BLOCK, 0, s>>>(pl.plain, part);
    k_force_step<<<pl.grid_flat, BLOCK, 0, s>>>(pl.plain, KIND_LP, 0, locked);
    launch_gain(pl, s);
    launch_after(pl, s);
    k_lp_outputs<<<pl.grid_flat, BLOCK, 0, s>>>(pl.plain, inX, move);
    JET_TRY(hipGetLastError());
    JET_TRY(stream_wait(ctx, s));
    return JET_OK;
}

extern "C" int jet_rebalance_step(jet_context *ctx, const jet_csr *g, const jet_params *params,
                                  const int32_t *part, int32_t kind, int32_t t, int32_t *dest, int64_t *loss,
                                  int32_t *slot, void *stream)
{
    if (!ctx || !g || !params) return JET_EINVAL;
    int st = check_params(g, params);
    if (st) return st;
    if (kind != KIND_RW && kind != KIND_RS) return JET_EINVAL;
    const int n = g->n;
    if (n > 0 && (!part || !dest || !loss || !slot)) return JET_EINVAL;
    if (params->k < 2 || t < 0) return JET_EINVAL;
    if (n == 0) return JET_OK;
    hipStream_t s = (hipStream_t)stream;
    JET_TRY(hipSetDevice(ctx->device));
    int32_t *pdv = (int32_t *)ws_get(ctx, WS_DBG_LOCK, sizeof(int32_t) * n);
    if (!pdv) return JET_ENOMEM;
    DebugOut dbg;
    dbg.loss = loss;
    dbg.slot = slot;
    dbg.pd = pdv;
    Launch L;
    Plan pl;
    st = step_setup(ctx, g, params, part, dbg, L, pl, s);
    if (st) return st;
    set_it(pl, 0);
    const KArgs &p = pl.plain;
    k_step_defaults<<<pl.grid_flat, BLOCK, 0, s>>>(p, part);
    k_force_step<<<1, BLOCK, 0, s>>>(p, kind, t, nullptr);
    launch_rb_loss(pl, s);
    launch_rb_cutoff(pl, s);
    launch_after(pl, s);
    launch_rb_select(pl, s);
    JET_TRY(hipGetLastError());
    JET_TRY(hipMemcpyAsync(dest, p.dest, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    JET_TRY(stream_wait(ctx, s));
    return JET_OK;
}
