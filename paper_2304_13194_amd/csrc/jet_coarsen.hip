// Multilevel scaffold on gfx950 (Algorithms 1 and 2): heavy-edge matching,
// hashed contraction, projection, a seeded random coarsest partition, and the
// driver that refines every level on the way back up.
//
// Heavy-edge matching runs in rounds of mutual proposals: every unmatched
// vertex proposes to the unmatched neighbour across its heaviest edge (ties
// to the smaller edge hash mix64(hseed ^ (min << 32 | max)), then to the
// smaller id) and mutual proposals match. A device-side check stops the
// rounds once a round matches fewer than 1% of the vertices, so the 16
// rounds are enqueued without host synchronisation. Pairs and singletons
// are numbered by their smaller member (exclusive scan over leader flags).
// Contraction follows Algorithm 2: an upper bound of each coarse row's length
// (sum of member degrees), an exclusive scan of the bounds, open-addressed
// per-row hash tables (twice the bound) filled with atomic CAS + add, and a
// compaction of the occupied slots. Coarse rows come out unsorted; nothing
// downstream depends on row order.
#include <hip/hip_runtime.h>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "jet_device.h"
#include "jet_internal.h"

namespace jet {

constexpr int CB = 256;   // block size of the coarsening kernels
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = CB * SCAN_ITEMS;

struct CState {
    int32_t stop;
    int32_t newly;
    int32_t bad;
    int32_t pad;
    int64_t wsum, ewsum;
};

// --------------------------------------------------------- input checks ---

__global__ __launch_bounds__(CB) void k_chk_vertices(int n, const int64_t *xadj, const int32_t *vw, CState *st)
{
    __shared__ int64_t s_red[CB / 64];
    int64_t ws = 0;
    int bad = 0;
    for (int v = blockIdx.x * CB + threadIdx.x; v < n; v += gridDim.x * CB) {
        const int x = vw ? vw[v] : 1;
        if (x < 1) bad = 1;
        if (xadj[v + 1] < xadj[v]) bad = 1;
        ws += x;
    }
    ws = block_sum<CB>(ws, s_red);
    if (bad) st->bad = 1;
    if (threadIdx.x == 0) atomicAdd((unsigned long long *)&st->wsum, (unsigned long long)ws);
}

// Neighbour-range, self-loop and weight checks and the total edge weight.
// Block b takes the entries of row-mark interval b, [b * MARK, (b + 1) *
// MARK). When the interval's rows fit in LDS, their offsets are staged there
// and the entries are read coalesced, each finding its row by a binary search
// in LDS; otherwise each thread takes runs of 16 entries and searches their
// first row between the two marks.
constexpr int CHK_ROWS = 2048;
__global__ __launch_bounds__(CB) void k_chk_edges(int n, int64_t nnz, const int64_t *xadj, const int32_t *adj,
                                                  const int32_t *ew, const int32_t *mark, int64_t nmark, CState *st)
{
    __shared__ int64_t s_red[CB / 64];
    __shared__ int64_t s_x[CHK_ROWS + 1];
    int64_t ews = 0;
    int bad = 0;
    for (int64_t blk = blockIdx.x; blk * MARK < nnz; blk += gridDim.x) {
        const int64_t e_lo = blk * MARK, e_hi = e_lo + MARK < nnz ? e_lo + MARK : nnz;
        // rows r_lo..r_hi hold the interval on well-formed offsets; both stay
        // in [0, n) on malformed ones (k_chk_vertices flags those)
        int r_lo = mark[blk];
        int r_hi = blk + 1 < nmark ? mark[blk + 1] : n - 1;
        if (r_hi > n - 1) r_hi = n - 1;
        if (r_lo > r_hi) r_lo = r_hi;
        const int nr = r_hi - r_lo + 1;
        if (nr <= CHK_ROWS) {
            for (int i = threadIdx.x; i <= nr; i += CB) s_x[i] = xadj[r_lo + i];
            __syncthreads();
            for (int64_t e = e_lo + threadIdx.x; e < e_hi; e += CB) {
                int lo = 0, hi = nr;  // largest lo with s_x[lo] <= e
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_x[mid] <= e) lo = mid;
                    else hi = mid;
                }
                const int v = r_lo + lo;
                const int u = adj[e];
                const int w = ew ? ew[e] : 1;
                if (u < 0 || u >= n || u == v || w < 1) bad = 1;
                else ews += w;
            }
            __syncthreads();
            continue;
        }
        constexpr int RUN = 16;
        for (int64_t e0 = e_lo + (int64_t)threadIdx.x * RUN; e0 < e_hi; e0 += (int64_t)CB * RUN) {
            const int64_t e1 = e0 + RUN < e_hi ? e0 + RUN : e_hi;
            int lo = r_lo, hi = r_hi + 1;  // largest lo with xadj[lo] <= e0
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (xadj[mid] <= e0) lo = mid;
                else hi = mid;
            }
            int u[RUN], w[RUN];
#pragma unroll
            for (int j = 0; j < RUN; j++) {
                const int64_t e = e0 + j;
                u[j] = e < e1 ? adj[e] : -1;
                w[j] = e < e1 ? (ew ? ew[e] : 1) : 1;
            }
            int v = lo;
            int64_t vend = xadj[v + 1];
#pragma unroll
            for (int j = 0; j < RUN; j++) {
                const int64_t e = e0 + j;
                if (e >= e1) break;
                while (e >= vend && v < n - 1) {
                    v++;
                    vend = xadj[v + 1];
                }
                if (u[j] < 0 || u[j] >= n || u[j] == v || w[j] < 1) {
                    bad = 1;
                    continue;
                }
                ews += w[j];
            }
        }
    }
    ews = block_sum<CB>(ews, s_red);
    if (bad) st->bad = 1;
    if (threadIdx.x == 0) atomicAdd((unsigned long long *)&st->ewsum, (unsigned long long)ews);
}

// ---------------------------------------------------------------- scans ---

// Exclusive scan of int32 `in[0..n)` into int64 `out[0..n]` (out[n] = total).
__global__ __launch_bounds__(CB) void k_scan_tiles(const int32_t *in, int n, int64_t *tsum)
{
    __shared__ int64_t s_red[CB / 64];
    const int base = blockIdx.x * SCAN_TILE;
    int64_t acc = 0;
    for (int i = threadIdx.x; i < SCAN_TILE; i += CB) {
        const int j = base + i;
        if (j < n) acc += in[j];
    }
    acc = block_sum<CB>(acc, s_red);
    if (threadIdx.x == 0) tsum[blockIdx.x] = acc;
}

__global__ __launch_bounds__(CB) void k_scan_top(int64_t *tsum, int ntiles)
{
    __shared__ int64_t s_scan[CB / 64];
    int64_t carry = 0;
    for (int base = 0; base < ntiles; base += CB) {
        const int i = base + threadIdx.x;
        const int64_t x = i < ntiles ? tsum[i] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan<CB>(x, s_scan, tot);
        if (i < ntiles) tsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) tsum[ntiles] = carry;
}

__global__ __launch_bounds__(CB) void k_scan_apply(const int32_t *in, int n, const int64_t *tsum, int64_t *out)
{
    __shared__ int64_t s_scan[CB / 64];
    const int base = blockIdx.x * SCAN_TILE;
    int64_t carry = tsum[blockIdx.x];
    for (int c = 0; c < SCAN_ITEMS; c++) {
        const int j = base + c * CB + threadIdx.x;
        const int64_t x = j < n ? in[j] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan<CB>(x, s_scan, tot);
        if (j < n) out[j] = carry + ex;
        carry += tot;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = tsum[gridDim.x];
}

static void scan_excl(const int32_t *in, int n, int64_t *out, int64_t *tsum, hipStream_t s)
{
    const int ntiles = std::max(1, (n + SCAN_TILE - 1) / SCAN_TILE);
    k_scan_tiles<<<ntiles, CB, 0, s>>>(in, n, tsum);
    k_scan_top<<<1, CB, 0, s>>>(tsum, ntiles);
    k_scan_apply<<<ntiles, CB, 0, s>>>(in, n, tsum, out);
}

// ------------------------------------------------------ heavy-edge match ---

// Larger is better: heavier edge, then smaller hash, then smaller id.
struct Prop {
    int32_t w;
    int32_t u;
    uint64_t h;
};
__device__ __forceinline__ bool prop_better(const Prop &a, const Prop &b)
{
    if (a.u < 0) return false;
    if (b.u < 0) return true;
    if (a.w != b.w) return a.w > b.w;
    if (a.h != b.h) return a.h < b.h;
    return a.u < b.u;
}

__device__ __forceinline__ Prop prop_shfl_xor(const Prop &p, int o, int width)
{
    Prop q;
    q.w = __shfl_xor(p.w, o, width);
    q.u = __shfl_xor(p.u, o, width);
    q.h = __shfl_xor(p.h, o, width);
    return q;
}

// taken[u] != 0: u is matched (a byte per vertex, so the gathers of the
// proposal rounds read a quarter of the bytes of the partner array)
__device__ __forceinline__ Prop prop_scan_row(int v, int64_t s, int64_t e, int lane, int stride, const int32_t *adj,
                                               const int32_t *ew, const uint8_t *taken, uint64_t hseed)
{
    // U entries per lane per round: their ids and weights, then their match
    // states, are loaded before any is examined
    constexpr int U = 8;
    Prop best{0, -1, 0};
    for (int64_t i0 = s + lane; i0 < e; i0 += (int64_t)stride * U) {
        int u[U], w[U], mu[U];
#pragma unroll
        for (int j = 0; j < U; j++) {
            const int64_t i = i0 + (int64_t)j * stride;
            u[j] = i < e ? adj[i] : -1;
            w[j] = i < e ? (ew ? ew[i] : 1) : 0;
        }
#pragma unroll
        for (int j = 0; j < U; j++) mu[j] = u[j] >= 0 ? taken[u[j]] : 1;
#pragma unroll
        for (int j = 0; j < U; j++) {
            if (u[j] < 0 || mu[j]) continue;
            const uint32_t lo = (uint32_t)(u[j] < v ? u[j] : v), hi = (uint32_t)(u[j] < v ? v : u[j]);
            Prop c{w[j], u[j], mix64(hseed ^ (((uint64_t)lo << 32) | hi))};
            if (prop_better(c, best)) best = c;
        }
    }
    return best;
}

// After the first round a vertex rescans its row only when last round's
// proposal has been matched since: the unmatched neighbours only shrink from
// round to round, so a proposal that is still unmatched is still the best,
// and a vertex that had no unmatched neighbour (-1) has none now.
__device__ __forceinline__ bool prop_stands(int round, const int32_t *prop, const uint8_t *taken, int v)
{
    if (round == 0) return false;
    const int pu = prop[v];
    return pu < 0 || !taken[pu];
}

// Proposals of the vertices of degree <= 64. Each lane of a wave first
// inspects one vertex with coalesced loads; only unmatched vertices whose
// proposal no longer stands are queued in LDS and scanned by the wave's
// groups of 8 lanes. Matched vertices cost no group time (k_hem_match clears
// their proposals once, when they match). Blocks b of nb.
__device__ __forceinline__ void propose_small(int b, int nb, int n, const int64_t *xadj, const int32_t *adj,
                                              const int32_t *ew, const int32_t *match, const uint8_t *taken,
                                              int32_t *prop, uint64_t hseed, int round, int32_t *s_q)
{
    constexpr int G = 8;
    const int lane = threadIdx.x & 63, gl = lane & (G - 1), grp = lane >> 3;
    int32_t *q = s_q + (threadIdx.x >> 6) * 64;
    const int nw = nb * (CB / 64);
    for (int64_t base = (int64_t)(b * (CB / 64) + (threadIdx.x >> 6)) * 64; base < n; base += (int64_t)nw * 64) {
        const int v = (int)base + lane;
        bool need = false;
        if (v < n) {
            const int64_t d = xadj[v + 1] - xadj[v];
            if (d <= 64 && match[v] < 0 && !prop_stands(round, prop, taken, v)) {
                if (d == 0) prop[v] = -1;  // no neighbour: nothing to scan
                else need = true;
            }
        }
        const uint64_t m = __ballot(need);
        if (need) q[__popcll(m & ((1ull << lane) - 1ull))] = v;
        lds_fence_wave();
        const int cnt = __popcll(m);
        for (int i = grp; i < cnt; i += 64 / G) {
            const int u = q[i];
            Prop r = prop_scan_row(u, xadj[u], xadj[u + 1], gl, G, adj, ew, taken, hseed);
#pragma unroll
            for (int o = G / 2; o > 0; o >>= 1) {
                Prop t = prop_shfl_xor(r, o, G);
                if (prop_better(t, r)) r = t;
            }
            if (gl == 0) prop[u] = r.u;
        }
        lds_fence_wave();
    }
}

// Rows of 65 to HEM_MID entries: one wave per row. The wave first inspects
// 64 list entries at once and queues the rows that need a scan.
__device__ __forceinline__ void propose_mid(int b, int nb, const int32_t *list, int cnt, const int64_t *xadj,
                                            const int32_t *adj, const int32_t *ew, const int32_t *match,
                                            const uint8_t *taken, int32_t *prop, uint64_t hseed, int round,
                                            int32_t *s_q)
{
    const int lane = threadIdx.x & 63;
    int32_t *q = s_q + (threadIdx.x >> 6) * 64;
    const int nw = nb * (CB / 64);
    for (int64_t base = (int64_t)(b * (CB / 64) + (threadIdx.x >> 6)) * 64; base < cnt; base += (int64_t)nw * 64) {
        const int i = (int)base + lane;
        int v = -1;
        bool need = false;
        if (i < cnt) {
            v = list[i];
            need = match[v] < 0 && !prop_stands(round, prop, taken, v);
        }
        const uint64_t m = __ballot(need);
        if (need) q[__popcll(m & ((1ull << lane) - 1ull))] = v;
        lds_fence_wave();
        const int nq = __popcll(m);
        for (int j = 0; j < nq; j++) {
            const int u = q[j];
            Prop r = prop_scan_row(u, xadj[u], xadj[u + 1], lane, 64, adj, ew, taken, hseed);
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                Prop t = prop_shfl_xor(r, o, 64);
                if (prop_better(t, r)) r = t;
            }
            if (lane == 0) prop[u] = r.u;
        }
        lds_fence_wave();
    }
}

// Rows of more than HEM_MID entries: one block per row.
__device__ __forceinline__ void propose_huge(int b, int nb, const int32_t *list, int cnt, const int64_t *xadj,
                                             const int32_t *adj, const int32_t *ew, const int32_t *match,
                                             const uint8_t *taken, int32_t *prop, uint64_t hseed, int round,
                                             Prop *s_p)
{
    for (int i = b; i < cnt; i += nb) {
        const int v = list[i];
        if (match[v] >= 0) continue;
        if (prop_stands(round, prop, taken, v)) continue;  // uniform over the block
        Prop r = prop_scan_row(v, xadj[v], xadj[v + 1], threadIdx.x, CB, adj, ew, taken, hseed);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            Prop t = prop_shfl_xor(r, o, 64);
            if (prop_better(t, r)) r = t;
        }
        if ((threadIdx.x & 63) == 0) s_p[threadIdx.x >> 6] = r;
        __syncthreads();
        if (threadIdx.x == 0) {
            Prop w = s_p[0];
            for (int k = 1; k < CB / 64; k++)
                if (prop_better(s_p[k], w)) w = s_p[k];
            prop[v] = w.u;
        }
        __syncthreads();
    }
}

// One launch per round for the three proposal roles, by block range: the
// rows of more than HEM_MID entries first (gh blocks, from the back of
// `big`), then those of 65 to HEM_MID (gm blocks, from its front), then every
// vertex of degree <= 64 (the remaining blocks). The roles touch disjoint
// vertices, and in one launch their tails overlap.
__global__ __launch_bounds__(CB) void k_hem_propose(int n, const int64_t *xadj, const int32_t *adj, const int32_t *ew,
                                                    const int32_t *match, const uint8_t *taken, int32_t *prop,
                                                    uint64_t hseed, const CState *st, int round,
                                                    const int32_t *mid, int nmid, const int32_t *huge, int nhuge,
                                                    int gh, int gm)
{
    __shared__ int32_t s_q[CB];
    __shared__ Prop s_p[CB / 64];
    if (st->stop) return;
    int b = blockIdx.x;
    if (b < gh) {
        propose_huge(b, gh, huge, nhuge, xadj, adj, ew, match, taken, prop, hseed, round, s_p);
        return;
    }
    b -= gh;
    if (b < gm) {
        propose_mid(b, gm, mid, nmid, xadj, adj, ew, match, taken, prop, hseed, round, s_q);
        return;
    }
    b -= gm;
    propose_small(b, (int)gridDim.x - gh - gm, n, xadj, adj, ew, match, taken, prop, hseed, round, s_q);
}

// Mutual proposals match; the smaller id of each pair writes both entries
// and clears both proposals, so that no later round sees a stale proposal
// of a matched vertex (the propose kernels skip matched vertices).
__global__ __launch_bounds__(CB) void k_hem_match(int n, int32_t *match, uint8_t *taken, int32_t *prop, CState *st)
{
    __shared__ int32_t s_red[CB / 64];
    if (st->stop) return;
    int cnt = 0;
    for (int v = blockIdx.x * CB + threadIdx.x; v < n; v += gridDim.x * CB) {
        if (match[v] >= 0) continue;
        const int u = prop[v];
        if (u > v && prop[u] == v) {
            match[v] = u;
            match[u] = v;
            taken[v] = 1;
            taken[u] = 1;
            prop[v] = -1;
            prop[u] = -1;
            cnt += 2;
        }
    }
    cnt = block_sum<CB>(cnt, s_red);
    if (threadIdx.x == 0 && cnt) atomicAdd(&st->newly, cnt);
}

__global__ void k_hem_round_end(int n, CState *st)
{
    if (st->stop) return;
    const int64_t newly = st->newly;
    if (newly == 0 || newly * 100 < (int64_t)n) st->stop = 1;
    st->newly = 0;
}

// Rows of more than 64 entries: those of at most HEM_MID entries (one wave
// each) from the front of `big`, the longer ones (one block each) from its
// back; counts in nbig[0] and nbig[1]. Each block counts its contiguous range
// first and takes its places with one atomic per list: a list counter is one
// address that every XCD reaches through memory, so one atomic per wave
// serialised into most of the kernel's time.
constexpr int HEM_MID = 1024;
__global__ __launch_bounds__(CB) void k_big_list(int n, const int64_t *xadj, int32_t *big, int32_t *nbig)
{
    __shared__ int32_t s_scan[CB / 64];
    __shared__ int32_t s_base[2];
    const int per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t l0 = (int64_t)blockIdx.x * per, h0 = l0 + per;
    const int lo = (int)(l0 < n ? l0 : n), hi = (int)(h0 < n ? h0 : n);
    int cm = 0, cl = 0;
    for (int v = lo + threadIdx.x; v < hi; v += CB) {
        const int64_t d = xadj[v + 1] - xadj[v];
        cm += d > 64 && d <= HEM_MID;
        cl += d > HEM_MID;
    }
    int totm, totl;
    const int offm = block_excl_scan<CB>(cm, s_scan, totm);
    const int offl = block_excl_scan<CB>(cl, s_scan, totl);
    if (threadIdx.x == 0) {
        s_base[0] = totm > 0 ? atomicAdd(&nbig[0], totm) : 0;
        s_base[1] = totl > 0 ? atomicAdd(&nbig[1], totl) : 0;
    }
    __syncthreads();
    int pm = s_base[0] + offm, pl = s_base[1] + offl;
    for (int v = lo + threadIdx.x; v < hi; v += CB) {
        const int64_t d = xadj[v + 1] - xadj[v];
        if (d > HEM_MID) big[n - 1 - pl++] = v;
        else if (d > 64) big[pm++] = v;
    }
}

// ------------------------------------------------------ two-hop matching ---
// Section 3.1: when heavy-edge matching leaves more than a quarter of the
// vertices unmatched, up to three passes match vertices two hops apart.
// Each pass gives every candidate a key; candidates of equal key are matched
// in ascending id order (first with second, third with fourth, ...):
//   leaves    (pass 0) unmatched, one entry: the neighbour;
//   twins     (pass 1) unmatched, 1 to 64 entries: a hash of the
//             neighbourhood (twins are relatives, so isolated vertices
//             never pair);
//   relatives (pass 2) unmatched, 1 to 64 entries: the matchmaker, the
//             smallest-id neighbour already matched with at most 1024
//             entries (hubs are never matchmakers).
// Non-candidates get TH_NONE and sort after every candidate (twin hashes
// keep 63 bits).
constexpr uint64_t TH_NONE = ~0ull;
constexpr int TH_MAXDEG = 64, TH_MM_MAXDEG = 1024;

__global__ __launch_bounds__(CB) void k_th_count(int n, const int32_t *match, int32_t *cnt)
{
    __shared__ int32_t s_red[CB / 64];
    int c = 0;
    for (int v = blockIdx.x * CB + threadIdx.x; v < n; v += gridDim.x * CB) c += match[v] < 0;
    c = block_sum<CB>(c, s_red);
    if (threadIdx.x == 0 && c) atomicAdd(cnt, c);
}

__global__ __launch_bounds__(CB) void k_th_keys(int n, int pass, const int64_t *xadj, const int32_t *adj,
                                                const int32_t *match, uint64_t *key, int32_t *val)
{
    for (int v = blockIdx.x * CB + threadIdx.x; v < n; v += gridDim.x * CB) {
        val[v] = v;
        uint64_t k = TH_NONE;
        const int64_t s = xadj[v];
        const int deg = (int)(xadj[v + 1] - s);
        if (match[v] < 0 && deg >= 1 && deg <= TH_MAXDEG) {
            if (pass == 0) {
                if (deg == 1) k = (uint64_t)(uint32_t)adj[s];
            } else if (pass == 1) {
                uint64_t h = 0;
                for (int e = 0; e < deg; e++) h += mix64((uint64_t)(uint32_t)adj[s + e] + 1);
                k = mix64(h ^ mix64((uint64_t)deg)) >> 1;
            } else {
                int mm = -1;
                for (int e = 0; e < deg; e++) {
                    const int u = adj[s + e];
                    if (match[u] < 0 || xadj[u + 1] - xadj[u] > TH_MM_MAXDEG) continue;
                    if (mm < 0 || u < mm) mm = u;
                }
                if (mm >= 0) k = (uint64_t)(uint32_t)mm;
            }
        }
        key[v] = k;
    }
}

// Start index of each sorted entry's run of equal keys (max-scanned next).
__global__ __launch_bounds__(CB) void k_th_runflag(int n, const uint64_t *key, int32_t *flag)
{
    for (int i = blockIdx.x * CB + threadIdx.x; i < n; i += gridDim.x * CB)
        flag[i] = (i == 0 || key[i] != key[i - 1]) ? i : 0;
}

__global__ __launch_bounds__(CB) void k_th_pair(int n, const uint64_t *key, const int32_t *val, const int32_t *run,
                                                int32_t *match)
{
    for (int i = blockIdx.x * CB + threadIdx.x; i + 1 < n; i += gridDim.x * CB) {
        const uint64_t k = key[i];
        if (k == TH_NONE || key[i + 1] != k || ((i - run[i]) & 1)) continue;
        const int a = val[i], b = val[i + 1];
        match[a] = b;
        match[b] = a;
    }
}

__global__ __launch_bounds__(CB) void k_leader_flags(int n, const int32_t *match, int32_t *flag)
{
    for (int v = blockIdx.x * CB + threadIdx.x; v < n; v += gridDim.x * CB) {
        const int m = match[v];
        flag[v] = (m < 0 || v < m) ? 1 : 0;
    }
}

// map[v] = coarse id of v's leader; coarse vertex weight and row-length bound
// are written by the leader.
__global__ __launch_bounds__(CB) void k_coarse_map(int n, const int32_t *match, const int64_t *cid,
                                                   const int64_t *xadj, const int32_t *vw, int32_t *map,
                                                   int32_t *cvw, int32_t *bound, int32_t *mem0, int32_t *mem1)
{
    for (int v = blockIdx.x * CB + threadIdx.x; v < n; v += gridDim.x * CB) {
        const int m = match[v];
        const bool leader = m < 0 || v < m;
        const int lead = leader ? v : m;
        const int c = (int)cid[lead];
        map[v] = c;
        if (leader) {
            int w = vw ? vw[v] : 1;
            int64_t b = xadj[v + 1] - xadj[v];
            if (m >= 0) {
                w += vw ? vw[m] : 1;
                b += xadj[m + 1] - xadj[m];
            }
            cvw[c] = w;
            bound[c] = (int32_t)b;
            mem0[c] = v;
            mem1[c] = m;
        }
    }
}

// Algorithm 2's insertOrLookup: every fine edge (v, u, w) with distinct coarse
// ends adds w to key map[u] in the table of row map[v]. Tables are open
// addressed over [toff[c], toff[c] + 2 * bound[c]) with linear probing.
__global__ __launch_bounds__(CB) void k_contract_insert(int n, int64_t nnz, const int64_t *xadj, const int32_t *adj,
                                                        const int32_t *ew, const int32_t *map, const int64_t *toff,
                                                        int32_t *tkey, int32_t *tval, int32_t *ccount)
{
    constexpr int RUN = 16;
    const int64_t nruns = (nnz + RUN - 1) / RUN;
    for (int64_t r = (int64_t)blockIdx.x * CB + threadIdx.x; r < nruns; r += (int64_t)gridDim.x * CB) {
        const int64_t e0 = r * RUN, e1 = e0 + RUN < nnz ? e0 + RUN : nnz;
        int lo = 0, hi = n;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (xadj[mid] <= e0) lo = mid; else hi = mid;
        }
        int v = lo;
        int64_t vend = xadj[v + 1];
        int cv = map[v];
        for (int64_t e = e0; e < e1; e++) {
            while (e >= vend) { v++; vend = xadj[v + 1]; cv = map[v]; }
            const int cu = map[adj[e]];
            if (cu == cv) continue;
            const int w = ew ? ew[e] : 1;
            const int64_t base = toff[cv];
            const uint32_t T = (uint32_t)(toff[cv + 1] - base);
            uint32_t h = ((uint32_t)cu * 2654435761u) % T;
            for (;;) {
                const int32_t old = atomicCAS(&tkey[base + h], -1, cu);
                if (old == -1) { atomicAdd(&ccount[cv], 1); atomicAdd(&tval[base + h], w); break; }
                if (old == cu) { atomicAdd(&tval[base + h], w); break; }
                h = h + 1 == T ? 0 : h + 1;
            }
        }
    }
}

// Compaction of each coarse row's occupied slots (8 lanes per row).
__global__ __launch_bounds__(CB) void k_contract_extract(int nc, const int64_t *toff, const int32_t *tkey,
                                                         const int32_t *tval, const int64_t *cxadj, int32_t *cadj,
                                                         int32_t *cew)
{
    constexpr int G = 8;
    const int gl = threadIdx.x & (G - 1);
    const int gshift = (threadIdx.x & 63) & ~(G - 1);
    const int ngroups = gridDim.x * (CB / G);
    const int nloop_rows = (nc + ngroups - 1) / ngroups;
    for (int it = 0; it < nloop_rows; it++) {
        const int c = it * ngroups + blockIdx.x * (CB / G) + (threadIdx.x >> 3);
        const bool rowok = c < nc;
        int64_t s = 0, e = 0, out = 0;
        if (rowok) { s = toff[c]; e = toff[c + 1]; out = cxadj[c]; }
        // lanes of a wave walk their rows in lockstep chunks of G slots
        int64_t len = e - s;
        int64_t maxlen = len;
        for (int o = 32; o > 0; o >>= 1) {
            int64_t y = __shfl_xor(maxlen, o, 64);
            maxlen = y > maxlen ? y : maxlen;
        }
        for (int64_t i = 0; i < maxlen; i += G) {
            const int64_t j = s + i + gl;
            const bool occ = rowok && i + gl < len && tkey[j] >= 0;
            const uint64_t m = __ballot(occ);
            const uint32_t gm = (uint32_t)((m >> gshift) & 0xFFu);
            if (occ) {
                const int pos = __popc(gm & ((1u << gl) - 1u));
                cadj[out + pos] = tkey[j];
                cew[out + pos] = tval[j];
            }
            out += __popc(gm);
        }
    }
}


// ---------------------------------------------------- LDS contraction ---
// Each coarse row is deduplicated in an LDS hash table (key = coarse
// neighbour, value = summed edge weight) built from its members' fine rows.
// A count pass sizes the rows, an exclusive scan places them, a fill pass
// writes them. Rows of bound <= 64 use 8-lane groups with 128 slots; rows of
// bound <= 512 one wave with 1024 slots; rows of bound <= 2048 one block with
// 4096 slots; larger rows a global table.
constexpr int CS_MAX = 64, CS_T = 128;
constexpr int CW_MAX = 512, CW_T = 1024;
constexpr int CM_MAX = 2048, CM_T = 4096;

__device__ __forceinline__ uint32_t chash(int key, int bits)
{
    return ((uint32_t)key * 2654435761u) >> (32 - bits);
}

// Fine entry idx (0 <= idx < d0 + d1) of the two member rows.
__device__ __forceinline__ int64_t member_entry(int64_t s0, int d0, int64_t s1, int idx)
{
    return idx < d0 ? s0 + idx : s1 + (idx - d0);
}

// Lists of the wave rows (count in cnt[3]), block rows (cnt[0]) and large
// rows (cnt[1]; their table slots, 2 * bound each, summed into ltot). Each
// block counts its contiguous stretch first and takes its places with one
// atomic per list (a list counter is one address for the whole device).
__global__ __launch_bounds__(CB) void k_cclass(int nc, const int32_t *bound, int32_t *listW, int32_t *listM,
                                               int32_t *listL, int32_t *cnt, int64_t *ltot)
{
    __shared__ int32_t s_scan[CB / 64];
    __shared__ int64_t s_red[CB / 64];
    __shared__ int32_t s_base[3];
    const int per = (nc + gridDim.x - 1) / gridDim.x;
    const int64_t l0 = (int64_t)blockIdx.x * per, h0 = l0 + per;
    const int lo = (int)(l0 < nc ? l0 : nc), hi = (int)(h0 < nc ? h0 : nc);
    int cw = 0, cm = 0, cl = 0;
    int64_t lw = 0;
    for (int c = lo + threadIdx.x; c < hi; c += CB) {
        const int b = bound[c];
        cw += b > CS_MAX && b <= CW_MAX;
        cm += b > CW_MAX && b <= CM_MAX;
        if (b > CM_MAX) {
            cl++;
            lw += 2 * (int64_t)b;
        }
    }
    int tw, tm, tl;
    const int ow = block_excl_scan<CB>(cw, s_scan, tw);
    const int om = block_excl_scan<CB>(cm, s_scan, tm);
    const int ol = block_excl_scan<CB>(cl, s_scan, tl);
    lw = block_sum<CB>(lw, s_red);
    if (threadIdx.x == 0) {
        s_base[0] = tw > 0 ? atomicAdd(&cnt[3], tw) : 0;
        s_base[1] = tm > 0 ? atomicAdd(&cnt[0], tm) : 0;
        s_base[2] = tl > 0 ? atomicAdd(&cnt[1], tl) : 0;
        if (lw) atomicAdd((unsigned long long *)ltot, (unsigned long long)lw);
    }
    __syncthreads();
    int pw = s_base[0] + ow, pm = s_base[1] + om, pl = s_base[2] + ol;
    for (int c = lo + threadIdx.x; c < hi; c += CB) {
        const int b = bound[c];
        if (b > CM_MAX) listL[pl++] = c;
        else if (b > CW_MAX) listM[pm++] = c;
        else if (b > CS_MAX) listW[pw++] = c;
    }
}

template <bool FILL>
__global__ __launch_bounds__(CB) void k_crow_small(int nc, const int32_t *bound, const int32_t *mem0,
                                                   const int32_t *mem1, const int64_t *xadj, const int32_t *adj,
                                                   const int32_t *ew, const int32_t *map, int32_t *ccount,
                                                   const int64_t *cxadj, int32_t *cadj, int32_t *cew,
                                                   int32_t *overflow)
{
    __shared__ int32_t keys[(CB / 8) * CS_T];
    __shared__ int32_t vals[(CB / 8) * CS_T];
    for (int i = threadIdx.x; i < (CB / 8) * CS_T; i += CB) { keys[i] = -1; vals[i] = 0; }
    __syncthreads();
    const int gl = threadIdx.x & 7;
    const int gshift = (threadIdx.x & 63) & ~7;
    int32_t *K = keys + (threadIdx.x >> 3) * CS_T;
    int32_t *V = vals + (threadIdx.x >> 3) * CS_T;
    const int ngroups = gridDim.x * (CB / 8);
    for (int c = blockIdx.x * (CB / 8) + (threadIdx.x >> 3); c < nc; c += ngroups) {
        if (bound[c] > CS_MAX) continue;
        const int m0 = mem0[c], m1 = mem1[c];
        const int64_t s0 = xadj[m0];
        const int d0 = (int)(xadj[m0 + 1] - s0);
        int64_t s1 = 0;
        int d1 = 0;
        if (m1 >= 0) { s1 = xadj[m1]; d1 = (int)(xadj[m1 + 1] - s1); }
        // at most CS_MAX = 64 member entries: 8 per lane, all loaded first
        int cuv[8], wv[8];
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const int idx = gl + q * 8;
            const int64_t e = member_entry(s0, d0, s1, idx);
            cuv[q] = idx < d0 + d1 ? adj[e] : -1;
            wv[q] = idx < d0 + d1 ? (ew ? ew[e] : 1) : 0;
        }
#pragma unroll
        for (int q = 0; q < 8; q++) cuv[q] = cuv[q] >= 0 ? map[cuv[q]] : -1;
        for (int q = 0; q < 8; q++) {
            const int cu = cuv[q];
            if (cu < 0 || cu == c) continue;
            const int w = wv[q];
            uint32_t h = chash(cu, 7);
            for (int probe = 0;; probe++) {
                if (probe == CS_T) { *overflow = 1; break; }  // cannot happen: <= 64 keys in 128 slots
                const int old = atomicCAS(&K[h], -1, cu);
                if (old == -1 || old == cu) { if (FILL) atomicAdd(&V[h], w); break; }
                h = (h + 1) & (CS_T - 1);
            }
        }
        lds_fence_wave();
        if (!FILL) {
            int cnt = 0;
            for (int j = gl; j < CS_T; j += 8) {
                if (K[j] >= 0) { cnt++; K[j] = -1; }
            }
            cnt = gsum<8>(cnt);
            if (gl == 0) ccount[c] = cnt;
        } else {
            int64_t out = cxadj[c];
            for (int j0 = 0; j0 < CS_T; j0 += 8) {
                const int j = j0 + gl;
                const int key = K[j];
                const bool occ = key >= 0;
                const uint32_t gm = (uint32_t)((__ballot(occ) >> gshift) & 0xFFu);
                if (occ) {
                    const int pos = __popc(gm & ((1u << gl) - 1u));
                    cadj[out + pos] = key;
                    cew[out + pos] = V[j];
                    K[j] = -1;
                    V[j] = 0;
                }
                out += __popc(gm);
            }
        }
        lds_fence_wave();
    }
}

template <bool FILL>
__global__ __launch_bounds__(CB) void k_crow_wave(const int32_t *list, int cntW, const int32_t *mem0,
                                                  const int32_t *mem1, const int64_t *xadj, const int32_t *adj,
                                                  const int32_t *ew, const int32_t *map, int32_t *ccount,
                                                  const int64_t *cxadj, int32_t *cadj, int32_t *cew,
                                                  int32_t *overflow)
{
    __shared__ int32_t keys[(CB / 64) * CW_T];
    __shared__ int32_t vals[(CB / 64) * CW_T];
    for (int i = threadIdx.x; i < (CB / 64) * CW_T; i += CB) { keys[i] = -1; vals[i] = 0; }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    int32_t *K = keys + (threadIdx.x >> 6) * CW_T;
    int32_t *V = vals + (threadIdx.x >> 6) * CW_T;
    constexpr int PER = CW_T / 64;
    const int nw = gridDim.x * (CB / 64);
    for (int r = blockIdx.x * (CB / 64) + (threadIdx.x >> 6); r < cntW; r += nw) {
        const int c = list[r];
        const int m0 = mem0[c], m1 = mem1[c];
        const int64_t s0 = xadj[m0];
        const int d0 = (int)(xadj[m0 + 1] - s0);
        int64_t s1 = 0;
        int d1 = 0;
        if (m1 >= 0) { s1 = xadj[m1]; d1 = (int)(xadj[m1 + 1] - s1); }
        // at most CW_MAX = 512 member entries: 8 per lane, all loaded first
        constexpr int UW = CW_MAX / 64;
        int cuv[UW], wv[UW];
#pragma unroll
        for (int q = 0; q < UW; q++) {
            const int idx = lane + q * 64;
            const int64_t e = member_entry(s0, d0, s1, idx);
            cuv[q] = idx < d0 + d1 ? adj[e] : -1;
            wv[q] = idx < d0 + d1 ? (ew ? ew[e] : 1) : 0;
        }
#pragma unroll
        for (int q = 0; q < UW; q++) cuv[q] = cuv[q] >= 0 ? map[cuv[q]] : -1;
        for (int q = 0; q < UW; q++) {
            const int cu = cuv[q];
            if (cu < 0 || cu == c) continue;
            const int w = wv[q];
            uint32_t h = chash(cu, 10);
            for (int probe = 0;; probe++) {
                if (probe == CW_T) { *overflow = 1; break; }  // cannot happen: <= 512 keys in 1024 slots
                const int old = atomicCAS(&K[h], -1, cu);
                if (old == -1 || old == cu) { if (FILL) atomicAdd(&V[h], w); break; }
                h = (h + 1) & (CW_T - 1);
            }
        }
        lds_fence_wave();
        int mine = 0;
        const int j0 = lane * PER;
        for (int q = 0; q < PER; q++) mine += K[j0 + q] >= 0;
        if (!FILL) {
            const int tot = gsum<64>(mine);
            if (lane == 0) ccount[c] = tot;
            for (int q = 0; q < PER; q++) K[j0 + q] = -1;
        } else {
            int64_t out = cxadj[c] + (wave_incl_scan(mine) - mine);
            for (int q = 0; q < PER; q++) {
                const int key = K[j0 + q];
                if (key >= 0) {
                    cadj[out] = key;
                    cew[out] = V[j0 + q];
                    out++;
                    K[j0 + q] = -1;
                    V[j0 + q] = 0;
                }
            }
        }
        lds_fence_wave();
    }
}

template <bool FILL>
__global__ __launch_bounds__(CB) void k_crow_medium(const int32_t *list, int cntM, const int32_t *mem0,
                                                    const int32_t *mem1, const int64_t *xadj, const int32_t *adj,
                                                    const int32_t *ew, const int32_t *map, int32_t *ccount,
                                                    const int64_t *cxadj, int32_t *cadj, int32_t *cew,
                                                    int32_t *overflow)
{
    extern __shared__ int32_t lds[];
    __shared__ int32_t s_red[CB / 64];
    constexpr int PER = CM_T / CB;
    int32_t *K = lds, *V = lds + CM_T;
    for (int i = threadIdx.x; i < CM_T; i += CB) { K[i] = -1; V[i] = 0; }
    __syncthreads();
    for (int r = blockIdx.x; r < cntM; r += gridDim.x) {
        const int c = list[r];
        const int m0 = mem0[c], m1 = mem1[c];
        const int64_t s0 = xadj[m0];
        const int d0 = (int)(xadj[m0 + 1] - s0);
        int64_t s1 = 0;
        int d1 = 0;
        if (m1 >= 0) { s1 = xadj[m1]; d1 = (int)(xadj[m1 + 1] - s1); }
        // at most CM_MAX = 2048 member entries: CM_MAX / CB per thread, all loaded first
        constexpr int UM = CM_MAX / CB;
        int cuv[UM], wv[UM];
#pragma unroll
        for (int q = 0; q < UM; q++) {
            const int idx = threadIdx.x + q * CB;
            const int64_t e = member_entry(s0, d0, s1, idx);
            cuv[q] = idx < d0 + d1 ? adj[e] : -1;
            wv[q] = idx < d0 + d1 ? (ew ? ew[e] : 1) : 0;
        }
#pragma unroll
        for (int q = 0; q < UM; q++) cuv[q] = cuv[q] >= 0 ? map[cuv[q]] : -1;
        for (int q = 0; q < UM; q++) {
            const int cu = cuv[q];
            if (cu < 0 || cu == c) continue;
            const int w = wv[q];
            uint32_t h = chash(cu, 12);
            for (int probe = 0;; probe++) {
                if (probe == CM_T) { *overflow = 1; break; }  // cannot happen: <= 2048 keys in 4096 slots
                const int old = atomicCAS(&K[h], -1, cu);
                if (old == -1 || old == cu) { if (FILL) atomicAdd(&V[h], w); break; }
                h = (h + 1) & (CM_T - 1);
            }
        }
        __syncthreads();
        int mine = 0;
        const int j0 = threadIdx.x * PER;
        for (int q = 0; q < PER; q++) mine += K[j0 + q] >= 0;
        if (!FILL) {
            const int tot = block_sum<CB>(mine, s_red);
            if (threadIdx.x == 0) ccount[c] = tot;
            for (int q = 0; q < PER; q++) K[j0 + q] = -1;
        } else {
            int tot;
            int64_t out = cxadj[c] + block_excl_scan<CB>(mine, s_red, tot);
            for (int q = 0; q < PER; q++) {
                const int key = K[j0 + q];
                if (key >= 0) {
                    cadj[out] = key;
                    cew[out] = V[j0 + q];
                    out++;
                    K[j0 + q] = -1;
                    V[j0 + q] = 0;
                }
            }
        }
        __syncthreads();
    }
}

// Large coarse rows (more than CM_MAX member entries) are spread over the
// grid: the member entries in chunks of LCC per block for the insertion, the
// row's table in chunks of LTC slots per block for the extraction, so a hub
// no longer waits on one block. A table slot holds (key << 32) | weight sum,
// or LEMPTY; insertions race only on slot placement, and rows are compared
// and used as sets (every consumer is independent of the order of a row's
// entries).
constexpr int LCC = 4096;
constexpr int LTC = 4096;
constexpr uint64_t LEMPTY = ~0ull;

// Exclusive scans over the large rows (single block): table offsets (2 *
// bound slots each), insertion chunks and extraction chunks; also zeroes the
// rows' distinct-key counts and output cursors.
__global__ __launch_bounds__(CB) void k_cl_offsets(const int32_t *listL, int cntL, const int32_t *bound, int64_t *toffL,
                                                   int32_t *ich, int32_t *ech, int32_t *ccount, int32_t *cur)
{
    __shared__ int64_t s_scan[CB / 64];
    __shared__ int32_t s_scan32[CB / 64];
    int64_t carry = 0;
    int32_t ci = 0, ce = 0;
    for (int base = 0; base < cntL; base += CB) {
        const int i = base + threadIdx.x;
        const int b = i < cntL ? bound[listL[i]] : 0;
        const int64_t x = 2 * (int64_t)b;
        int64_t tot;
        const int64_t ex = block_excl_scan<CB>(x, s_scan, tot);
        int32_t ti, te;
        const int32_t exi = block_excl_scan<CB>((int32_t)((b + LCC - 1) / LCC), s_scan32, ti);
        const int32_t exe = block_excl_scan<CB>((int32_t)((x + LTC - 1) / LTC), s_scan32, te);
        if (i < cntL) {
            toffL[i] = carry + ex;
            ich[i] = ci + exi;
            ech[i] = ce + exe;
            ccount[listL[i]] = 0;
            cur[i] = 0;
        }
        carry += tot;
        ci += ti;
        ce += te;
    }
    if (threadIdx.x == 0) {
        toffL[cntL] = carry;
        ich[cntL] = ci;
        ech[cntL] = ce;
    }
}

// Largest r in [0, cnt) with off[r] <= x (off[0] = 0 <= x).
__device__ __forceinline__ int chunk_row(const int32_t *off, int cnt, int x)
{
    int lo = 0, hi = cnt;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Insertion: one block per chunk of LCC member entries of a large row, into
// the row's global open-addressed table of 2 * bound slots; the distinct
// keys a block claims are added to the row's count.
__global__ __launch_bounds__(CB) void k_crow_large_insert(const int32_t *listL, int cntL, const int64_t *toffL,
                                                          const int32_t *ich, const int32_t *mem0, const int32_t *mem1,
                                                          const int64_t *xadj, const int32_t *adj, const int32_t *ew,
                                                          const int32_t *map, unsigned long long *tab,
                                                          int32_t *ccount, int32_t *overflow)
{
    __shared__ int32_t s_red[CB / 64];
    constexpr int U = LCC / CB;
    const int nch = ich[cntL];
    for (int ci = blockIdx.x; ci < nch; ci += gridDim.x) {
        const int r = chunk_row(ich, cntL, ci);
        const int c = listL[r];
        const int m0 = mem0[c], m1 = mem1[c];
        const int64_t base = toffL[r];
        const uint32_t T = (uint32_t)(toffL[r + 1] - base);
        const int64_t s0 = xadj[m0];
        const int d0 = (int)(xadj[m0 + 1] - s0);
        int64_t s1 = 0;
        int d1 = 0;
        if (m1 >= 0) { s1 = xadj[m1]; d1 = (int)(xadj[m1 + 1] - s1); }
        const int lo = (ci - ich[r]) * LCC, hi = min(lo + LCC, d0 + d1);
        int cu[U], w[U];
#pragma unroll
        for (int q = 0; q < U; q++) {
            const int idx = lo + q * CB + threadIdx.x;
            const int64_t e = member_entry(s0, d0, s1, idx);
            cu[q] = idx < hi ? adj[e] : -1;
            w[q] = idx < hi ? (ew ? ew[e] : 1) : 0;
        }
#pragma unroll
        for (int q = 0; q < U; q++) cu[q] = cu[q] >= 0 ? map[cu[q]] : -1;
        int claimed = 0;
        for (int q = 0; q < U; q++) {
            if (cu[q] < 0 || cu[q] == c) continue;
            const unsigned long long want = ((unsigned long long)(uint32_t)cu[q] << 32) | (uint32_t)w[q];
            uint32_t h = ((uint32_t)cu[q] * 2654435761u) % T;
            for (uint32_t probe = 0;; probe++) {
                if (probe == T) { *overflow = 1; break; }  // cannot happen: <= bound keys in 2 * bound slots
                const unsigned long long old = atomicCAS(&tab[base + h], (unsigned long long)LEMPTY, want);
                if (old == LEMPTY) { claimed++; break; }
                // coarse edge weights stay below 2^31 (multilevel limit): no carry into the key
                if ((uint32_t)(old >> 32) == (uint32_t)cu[q]) { atomicAdd(&tab[base + h], (unsigned long long)(uint32_t)w[q]); break; }
                h = h + 1 == T ? 0 : h + 1;
            }
        }
        const int tot = block_sum<CB>(claimed, s_red);
        if (threadIdx.x == 0 && tot) atomicAdd(&ccount[c], tot);
    }
}

// Extraction: one block per chunk of LTC table slots of a large row; each
// wave appends its occupied slots at the row's cursor.
__global__ __launch_bounds__(CB) void k_crow_large_extract(const int32_t *listL, int cntL, const int64_t *toffL,
                                                           const int32_t *ech, const unsigned long long *tab,
                                                           int32_t *cur, const int64_t *cxadj, int32_t *cadj,
                                                           int32_t *cew)
{
    constexpr int U = LTC / CB;
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    const int nch = ech[cntL];
    for (int ci = blockIdx.x; ci < nch; ci += gridDim.x) {
        const int r = chunk_row(ech, cntL, ci);
        const int c = listL[r];
        const int64_t base = toffL[r], T = toffL[r + 1] - base;
        const int64_t j0 = (int64_t)(ci - ech[r]) * LTC;
        unsigned long long v[U];
        int cnt = 0;
#pragma unroll
        for (int q = 0; q < U; q++) {
            const int64_t j = j0 + q * CB + threadIdx.x;
            v[q] = j < T ? tab[base + j] : LEMPTY;
            cnt += __popcll(__ballot(v[q] != LEMPTY));
        }
        int wbase = 0;
        if (lane == 0 && cnt) wbase = atomicAdd(&cur[r], cnt);
        wbase = __shfl(wbase, 0, 64);
        const int64_t out = cxadj[c] + wbase;
        int pos = 0;
#pragma unroll
        for (int q = 0; q < U; q++) {
            const bool occ = v[q] != LEMPTY;
            const uint64_t m = __ballot(occ);
            if (occ) {
                const int64_t o = out + pos + __popcll(m & below);
                cadj[o] = (int32_t)(v[q] >> 32);
                cew[o] = (int32_t)(uint32_t)v[q];
            }
            pos += __popcll(m);
        }
    }
}

__global__ __launch_bounds__(CB) void k_double(const int32_t *b, int32_t *b2, int m)
{
    for (int i = blockIdx.x * CB + threadIdx.x; i < m; i += gridDim.x * CB) b2[i] = 2 * b[i];
}

__global__ __launch_bounds__(CB) void k_project(int n, const int32_t *map, const int32_t *pc, int32_t *pf)
{
    for (int v = blockIdx.x * CB + threadIdx.x; v < n; v += gridDim.x * CB) pf[v] = pc[map[v]];
}

// Seeded uniform random part per vertex: floor(stream(seed, v) * k / 2^64).
__global__ __launch_bounds__(CB) void k_random_part(int n, int k, uint64_t seed, int32_t *p)
{
    for (int v = blockIdx.x * CB + threadIdx.x; v < n; v += gridDim.x * CB)
        p[v] = (int32_t)__umul64hi(stream64(seed, (uint64_t)v), (uint64_t)k);
}

// ----------------------------------------------------------------- host ---

#define JET_TRY(expr)                                      \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return hip_status(ctx, e_);  \
    } while (0)

static int grid_for(const jet_context *ctx, int64_t items, int per_block, int cap_mult = 8)
{
    int64_t b = (items + per_block - 1) / per_block;
    b = std::max<int64_t>(1, std::min<int64_t>(b, (int64_t)ctx->num_cu * cap_mult));
    return (int)b;
}

// Cheap checks every entry point runs before kernels index through the graph.
int check_graph(jet_context *ctx, const jet_csr *g, uint32_t flags, hipStream_t s)
{
    if (g->n < 0 || g->nnz < 0) return JET_EGRAPH;
    if (g->n == 0) return JET_OK;
    if (!g->xadj || (g->nnz > 0 && !g->adjncy)) return JET_EINVAL;
    if (flags & JET_F_VALIDATE) {
        int st = validate_full_csr(ctx, g, s);
        if (st) return st;
    }
    CState *st = (CState *)ws_get(ctx, WS_H1, sizeof(CState));
    if (!st) return JET_ENOMEM;
    JET_TRY(hipMemsetAsync(st, 0, sizeof(CState), s));
    int64_t *ends = (int64_t *)((char *)ctx->pinned + 2048);
    JET_TRY(hipMemcpyAsync(ends, g->xadj, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    JET_TRY(hipMemcpyAsync(ends + 1, g->xadj + g->n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    JET_TRY(stream_wait(ctx, s));
    if (ends[0] != 0 || ends[1] != g->nnz) return JET_EGRAPH;
    k_chk_vertices<<<grid_for(ctx, g->n, CB, 4), CB, 0, s>>>(g->n, g->xadj, g->vwgt, st);
    if (g->nnz > 0) {
        int32_t *mark = nullptr;
        int64_t nmark = 0;
        const int rs = row_marks(ctx, g->xadj, g->n, g->nnz, &mark, &nmark, s);
        if (rs) return rs;
        k_chk_edges<<<grid_for(ctx, (g->nnz + MARK - 1) / MARK, 1), CB, 0, s>>>(g->n, g->nnz, g->xadj, g->adjncy,
                                                                              g->adjwgt, mark, nmark, st);
    }
    JET_TRY(hipGetLastError());
    CState *h = (CState *)((char *)ctx->pinned + 2304);
    JET_TRY(hipMemcpyAsync(h, st, sizeof(CState), hipMemcpyDeviceToHost, s));
    JET_TRY(stream_wait(ctx, s));
    if (h->bad) return JET_EGRAPH;
    if (h->wsum >= ((int64_t)1 << 31) || h->ewsum >= ((int64_t)1 << 31)) return JET_EOVERFLOW;
    return JET_OK;
}

void *jet::Arena::alloc(size_t bytes)
{
    bytes = (std::max<size_t>(bytes, 16) + 255) & ~(size_t)255;
    while (cur < chunks.size()) {
        if (used + bytes <= chunks[cur].bytes) {
            void *p = (char *)chunks[cur].ptr + used;
            used += bytes;
            return p;
        }
        cur++;
        used = 0;
    }
    size_t total = 0;
    for (const Buffer &b : chunks) total += b.bytes;
    Buffer b;
    b.bytes = std::max<size_t>({bytes, total, (size_t)64 << 20});
    if (hipMalloc(&b.ptr, b.bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    chunks.push_back(b);
    cur = chunks.size() - 1;
    used = bytes;
    return b.ptr;
}

// Only between calls (nothing queued still uses the memory).
void jet::Arena::reset()
{
    if (chunks.size() > 1) {
        size_t total = 0;
        for (const Buffer &b : chunks) total += b.bytes;
        release();
        Buffer b;
        if (hipMalloc(&b.ptr, total) == hipSuccess) {
            b.bytes = total;
            chunks.push_back(b);
        } else {
            (void)hipGetLastError();
        }
    }
    cur = 0;
    used = 0;
}

void jet::Arena::release()
{
    for (Buffer &b : chunks)
        if (b.ptr) (void)hipFree(b.ptr);
    chunks.clear();
    cur = 0;
    used = 0;
}

static void *hier_alloc(jet_hierarchy *h, size_t bytes)
{
    if (h->arena) return h->arena->alloc(bytes);
    void *p = nullptr;
    if (h->pool) {
        if (hipMallocFromPoolAsync(&p, bytes ? bytes : 16, h->pool, h->pool_stream) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        h->owned.push_back(p);
        return p;
    }
    if (hipMalloc(&p, bytes ? bytes : 16) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    h->owned.push_back(p);
    return p;
}

static void hier_release(jet_hierarchy *h)
{
    if (h->arena) h->arena->reset();
    for (void *p : h->owned) {
        if (h->pool) (void)hipFreeAsync(p, h->pool_stream);
        else (void)hipFree(p);
    }
    h->owned.clear();
}

// Two-hop passes while more than n/4 vertices are unmatched (one count and
// wait per pass).
static int two_hop(jet_context *ctx, const jet_csr *f, int32_t *match, hipStream_t s)
{
    const int n = f->n;
    if (n == 0) return JET_OK;
    const size_t nn = (size_t)n;
    int32_t *cnt = (int32_t *)ws_get(ctx, WS_TH_RUN, nn * 8 + 64);
    int32_t *flag = cnt + 16, *run = flag + nn;
    uint64_t *key = (uint64_t *)ws_get(ctx, WS_TH_KEY, nn * 16);
    int32_t *val = (int32_t *)ws_get(ctx, WS_TH_VAL, nn * 8);
    if (!cnt || !key || !val) return JET_ENOMEM;
    uint64_t *key2 = key + nn;
    int32_t *val2 = val + nn;
    size_t sort_bytes = 0, scan_bytes = 0;
    JET_TRY(rocprim::radix_sort_pairs(nullptr, sort_bytes, key, key2, val, val2, nn, 0, 64, s));
    JET_TRY(rocprim::inclusive_scan(nullptr, scan_bytes, flag, run, nn, rocprim::maximum<int32_t>(), s));
    void *tmp = ws_get(ctx, WS_TH_TMP, std::max(sort_bytes, scan_bytes) + 256);
    if (!tmp) return JET_ENOMEM;
    int32_t *hcnt = (int32_t *)((char *)ctx->pinned + 2560);
    const int gv = grid_for(ctx, n, CB, 4);
    for (int pass = 0; pass < 3; pass++) {
        JET_TRY(hipMemsetAsync(cnt, 0, 4, s));
        k_th_count<<<gv, CB, 0, s>>>(n, match, cnt);
        JET_TRY(hipMemcpyAsync(hcnt, cnt, 4, hipMemcpyDeviceToHost, s));
        JET_TRY(stream_wait(ctx, s));
        if (4 * (int64_t)*hcnt <= (int64_t)n) break;
        k_th_keys<<<gv, CB, 0, s>>>(n, pass, f->xadj, f->adjncy, match, key, val);
        size_t b = sort_bytes;
        JET_TRY(rocprim::radix_sort_pairs(tmp, b, key, key2, val, val2, nn, 0, 64, s));
        k_th_runflag<<<gv, CB, 0, s>>>(n, key2, flag);
        b = scan_bytes;
        JET_TRY(rocprim::inclusive_scan(tmp, b, flag, run, nn, rocprim::maximum<int32_t>(), s));
        k_th_pair<<<gv, CB, 0, s>>>(n, key2, val2, run, match);
        JET_TRY(hipGetLastError());
    }
    return JET_OK;
}

// One coarsening step of level graph f into c (device buffers owned by h).
// Returns the coarse vertex count in *nc_out (== f->n when nothing matched).
static int coarsen_level(jet_context *ctx, jet_hierarchy *h, const jet_csr *f, int level, uint64_t seed, bool th,
                         jet_csr *c, int32_t **map_out, int *nc_out, hipStream_t s)
{
    const int n = f->n;
    const size_t nn = (size_t)std::max(n, 1);
    int32_t *match = (int32_t *)ws_get(ctx, WS_C0, nn * 4);
    int32_t *prop = (int32_t *)ws_get(ctx, WS_C1, nn * 4);
    int32_t *big = (int32_t *)ws_get(ctx, WS_C2, nn * 4);
    int64_t *cid = (int64_t *)ws_get(ctx, WS_C3, (nn + 1) * 8);
    int64_t *tsum = (int64_t *)ws_get(ctx, WS_C4, ((nn + SCAN_TILE - 1) / SCAN_TILE + 2) * 8);
    CState *st = (CState *)ws_get(ctx, WS_H1, sizeof(CState) + 16);
    int32_t *nbig = (int32_t *)(st + 1);
    uint8_t *taken = (uint8_t *)ws_get(ctx, WS_C13, nn);
    if (!match || !prop || !big || !cid || !tsum || !st || !taken) return JET_ENOMEM;
    JET_TRY(hipMemsetAsync(match, 0xFF, nn * 4, s));
    JET_TRY(hipMemsetAsync(taken, 0, nn, s));
    JET_TRY(hipMemsetAsync(st, 0, sizeof(CState) + 16, s));
    const int gv = grid_for(ctx, n, CB, 4);
    k_big_list<<<gv, CB, 0, s>>>(n, f->xadj, big, nbig);
    int32_t *hbig = (int32_t *)((char *)ctx->pinned + 2400);
    JET_TRY(hipMemcpyAsync(hbig, nbig, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    JET_TRY(stream_wait(ctx, s));
    const int nmid = hbig[0], nhuge = hbig[1];
    const uint64_t hseed = stream64(seed, (uint64_t)(uint32_t)level);
    const int gs = grid_for(ctx, n, CB / 8);
    const int gh = nhuge > 0 ? std::min(nhuge, ctx->num_cu * 8) : 0;
    const int gm = nmid > 0 ? std::min((nmid + CB - 1) / CB, ctx->num_cu * 8) : 0;
    for (int round = 0; round < 16; round++) {
        k_hem_propose<<<gh + gm + gs, CB, 0, s>>>(n, f->xadj, f->adjncy, f->adjwgt, match, taken, prop, hseed, st,
                                                  round, big, nmid, big + (n - nhuge), nhuge, gh, gm);
        k_hem_match<<<gv, CB, 0, s>>>(n, match, taken, prop, st);
        k_hem_round_end<<<1, 1, 0, s>>>(n, st);
    }
    if (th) {
        const int st2 = two_hop(ctx, f, match, s);
        if (st2) return st2;
    }
    // coarse ids: leaders numbered in vertex order
    int32_t *flag = prop;  // proposals are no longer needed
    k_leader_flags<<<gv, CB, 0, s>>>(n, match, flag);
    scan_excl(flag, n, cid, tsum, s);
    int64_t *hn = (int64_t *)((char *)ctx->pinned + 2432);
    JET_TRY(hipMemcpyAsync(hn, cid + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    JET_TRY(stream_wait(ctx, s));
    const int nc = (int)*hn;
    *nc_out = nc;
    // a matching that keeps more than 90% of the vertices makes no level
    if (nc == n || 10 * (int64_t)nc > 9 * (int64_t)n) return JET_OK;
    const size_t ncc = (size_t)std::max(nc, 1);
    int32_t *map = (int32_t *)hier_alloc(h, nn * 4);
    int32_t *cvw = (int32_t *)hier_alloc(h, ncc * 4);
    int32_t *bound = (int32_t *)ws_get(ctx, WS_C5, ncc * 4);
    int32_t *ccount = (int32_t *)ws_get(ctx, WS_C7, ncc * 4);
    int32_t *mem0 = (int32_t *)ws_get(ctx, WS_C8, ncc * 4);
    int32_t *mem1 = (int32_t *)ws_get(ctx, WS_C9, ncc * 4);
    const size_t nce = (ncc + 1) & ~(size_t)1;  // even, so that the counters after the lists are 8-byte aligned
    int32_t *lists = (int32_t *)ws_get(ctx, WS_C12, 3 * nce * 4 + 64);
    int64_t *cxadj = (int64_t *)hier_alloc(h, (ncc + 1) * 8);
    if (!map || !cvw || !bound || !ccount || !mem0 || !mem1 || !lists || !cxadj) return JET_ENOMEM;
    int32_t *listM = lists, *listL = lists + nce, *listW = lists + 2 * nce;
    int32_t *ccnt = lists + 3 * nce;          // [0] block rows, [1] large rows, [2] probe overflow, [3] wave rows
    int64_t *ltot = (int64_t *)(ccnt + 4);    // table slots of the large rows (bytes 16..23)
    k_coarse_map<<<gv, CB, 0, s>>>(n, match, cid, f->xadj, f->vwgt, map, cvw, bound, mem0, mem1);
    JET_TRY(hipMemsetAsync(ccnt, 0, 64, s));
    k_cclass<<<grid_for(ctx, nc, CB, 4), CB, 0, s>>>(nc, bound, listW, listM, listL, ccnt, ltot);
    int32_t *hc = (int32_t *)((char *)ctx->pinned + 2448);
    JET_TRY(hipMemcpyAsync(hc, ccnt, 24, hipMemcpyDeviceToHost, s));
    JET_TRY(stream_wait(ctx, s));
    const int nM = hc[0], nL = hc[1], nW = hc[3];
    const int64_t lslots = *(int64_t *)(hc + 4);
    int64_t *toffL = nullptr;
    unsigned long long *ltab = nullptr;
    int32_t *ich = nullptr, *ech = nullptr, *lcur = nullptr;
    if (nL > 0) {
        toffL = (int64_t *)ws_get(ctx, WS_C6, ((size_t)nL + 1) * 8);
        ltab = (unsigned long long *)ws_get(ctx, WS_C10, (size_t)lslots * 8);
        ich = (int32_t *)ws_get(ctx, WS_C11, ((size_t)nL + 1) * 4 * 3);
        if (!toffL || !ltab || !ich) return JET_ENOMEM;
        ech = ich + nL + 1;
        lcur = ech + nL + 1;
        JET_TRY(hipMemsetAsync(ltab, 0xFF, (size_t)lslots * 8, s));
        k_cl_offsets<<<1, CB, 0, s>>>(listL, nL, bound, toffL, ich, ech, ccount, lcur);
        // the hub rows' insertion (bound by device-scope atomics) runs on the
        // second stream beside the LDS-table rows (bound by gathers); the two
        // touch disjoint coarse rows, and the scan below waits for both
        JET_TRY(hipEventRecord(ctx->fork_ev, s));
        JET_TRY(hipStreamWaitEvent(ctx->aux, ctx->fork_ev, 0));
        k_crow_large_insert<<<ctx->num_cu * 4, CB, 0, ctx->aux>>>(listL, nL, toffL, ich, mem0, mem1, f->xadj,
                                                                   f->adjncy, f->adjwgt, map, ltab, ccount, ccnt + 2);
    }
    const int gsmall = grid_for(ctx, nc, CB / 8);
    const size_t lds_m = 2 * CM_T * sizeof(int32_t);
    k_crow_small<false><<<gsmall, CB, 0, s>>>(nc, bound, mem0, mem1, f->xadj, f->adjncy, f->adjwgt, map, ccount,
                                               nullptr, nullptr, nullptr, ccnt + 2);
    const int gwave = std::max(1, std::min((nW + CB / 64 - 1) / (CB / 64), ctx->num_cu * 8));
    if (nW > 0)
        k_crow_wave<false><<<gwave, CB, 0, s>>>(listW, nW, mem0, mem1, f->xadj, f->adjncy, f->adjwgt, map, ccount,
                                                 nullptr, nullptr, nullptr, ccnt + 2);
    if (nM > 0)
        k_crow_medium<false><<<std::min(nM, ctx->num_cu * 4), CB, lds_m, s>>>(
            listM, nM, mem0, mem1, f->xadj, f->adjncy, f->adjwgt, map, ccount, nullptr, nullptr, nullptr, ccnt + 2);
    if (nL > 0) {
        JET_TRY(hipEventRecord(ctx->join_ev, ctx->aux));
        JET_TRY(hipStreamWaitEvent(s, ctx->join_ev, 0));
    }
    scan_excl(ccount, nc, cxadj, tsum, s);
    JET_TRY(hipMemcpyAsync(hn, cxadj + nc, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    JET_TRY(hipMemcpyAsync(hc, ccnt, 24, hipMemcpyDeviceToHost, s));
    JET_TRY(stream_wait(ctx, s));
    if (hc[2]) return JET_EHIP;  // a probe ran past its table: internal error
    const int64_t cnnz = *hn;
    int32_t *cadj = (int32_t *)hier_alloc(h, (size_t)std::max<int64_t>(cnnz, 1) * 4);
    int32_t *cew = (int32_t *)hier_alloc(h, (size_t)std::max<int64_t>(cnnz, 1) * 4);
    if (!cadj || !cew) return JET_ENOMEM;
    if (nL > 0) {
        // the hub rows' extraction beside the other rows' fill, as in the count pass
        JET_TRY(hipEventRecord(ctx->fork_ev, s));
        JET_TRY(hipStreamWaitEvent(ctx->aux, ctx->fork_ev, 0));
        k_crow_large_extract<<<ctx->num_cu * 4, CB, 0, ctx->aux>>>(listL, nL, toffL, ech, ltab, lcur, cxadj, cadj,
                                                                    cew);
    }
    k_crow_small<true><<<gsmall, CB, 0, s>>>(nc, bound, mem0, mem1, f->xadj, f->adjncy, f->adjwgt, map, ccount,
                                              cxadj, cadj, cew, ccnt + 2);
    if (nW > 0)
        k_crow_wave<true><<<gwave, CB, 0, s>>>(listW, nW, mem0, mem1, f->xadj, f->adjncy, f->adjwgt, map, ccount,
                                                cxadj, cadj, cew, ccnt + 2);
    if (nM > 0)
        k_crow_medium<true><<<std::min(nM, ctx->num_cu * 4), CB, lds_m, s>>>(
            listM, nM, mem0, mem1, f->xadj, f->adjncy, f->adjwgt, map, ccount, cxadj, cadj, cew, ccnt + 2);
    if (nL > 0) {
        JET_TRY(hipEventRecord(ctx->join_ev, ctx->aux));
        JET_TRY(hipStreamWaitEvent(s, ctx->join_ev, 0));
    }
    JET_TRY(hipGetLastError());
    c->n = nc;
    c->reserved = 0;
    c->nnz = cnnz;
    c->xadj = cxadj;
    c->adjncy = cadj;
    c->vwgt = cvw;
    c->adjwgt = cew;
    *map_out = map;
    return JET_OK;
}

static int build_hierarchy(jet_context *ctx, const jet_csr *g, const jet_params *prm, jet_hierarchy *h,
                           hipStream_t s)
{
    static std::once_flag attr;
    std::call_once(attr, [] {
        (void)hipFuncSetAttribute((const void *)k_crow_medium<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  65536);
        (void)hipFuncSetAttribute((const void *)k_crow_medium<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  65536);
    });
    h->device = ctx->device;
    h->lv.clear();
    h->maps.clear();
    h->lv.push_back(*g);
    const int64_t target = 8 * (int64_t)prm->k;
    while ((int)h->lv.size() < 64 && h->lv.back().n > target) {
        jet_csr f = h->lv.back();
        jet_csr c;
        int32_t *map = nullptr;
        int nc = 0;
        int st = coarsen_level(ctx, h, &f, (int)h->lv.size() - 1, prm->seed, (prm->flags & JET_F_TWO_HOP) != 0, &c,
                               &map, &nc, s);
        if (st) return st;
        // stall: the matching keeps more than 90% of the vertices (or matches
        // nothing), so the current level is the coarsest
        if (nc == f.n || 10 * (int64_t)nc > 9 * (int64_t)f.n) break;
        h->maps.push_back(map);
        h->lv.push_back(c);
    }
    h->maps.push_back(nullptr);
    h->nlevels = (int)h->lv.size();
    return JET_OK;
}

int hierarchy_build(jet_context *ctx, const jet_csr *g, const jet_params *prm, jet_hierarchy *h, hipStream_t s)
{
    return build_hierarchy(ctx, g, prm, h, s);
}

// ------------------------------------------------- graph-growing start --
// Coarsest-graph start (not the paper's, which takes Metis): vertices ordered
// by (smallest vertex id of their component, BFS distance from it, own id),
// the order cut into k runs of equal vertex weight. Each vertex's key
// (root << 32 | distance) starts at (v, 0) and is lowered to the smallest of
// its neighbours' keys plus one hop until a pass changes nothing; the only
// fixpoint of that rule is (component minimum, distance from it), so the
// order of the relaxation does not matter. A stable radix sort of the keys
// (values: vertex ids in id order) gives the order, a scan of the weights the
// runs.

__global__ __launch_bounds__(CB) void k_bfs_init(int n, uint64_t *key, int32_t *val)
{
    for (int v = blockIdx.x * CB + threadIdx.x; v < n; v += gridDim.x * CB) {
        key[v] = (uint64_t)(uint32_t)v << 32;
        val[v] = v;
    }
}

// One relaxation pass over the CSR entries in runs of 16 per thread (hub rows
// are spread over many threads): a run keeps the smallest neighbour key + 1
// of its current row and lowers the row's key with a 64-bit atomic minimum.
__device__ __forceinline__ void bfs_lower(uint64_t *key, int v, uint64_t m, bool &ch)
{
    if (m < key[v] && m < atomicMin((unsigned long long *)&key[v], (unsigned long long)m)) ch = true;
}

__global__ __launch_bounds__(CB) void k_bfs_relax(int n, int64_t nnz, const int64_t *xadj, const int32_t *adj,
                                                  uint64_t *key, int32_t *changed)
{
    constexpr int RUN = 16;
    bool ch = false;
    const int64_t nruns = (nnz + RUN - 1) / RUN;
    for (int64_t r = (int64_t)blockIdx.x * CB + threadIdx.x; r < nruns; r += (int64_t)gridDim.x * CB) {
        const int64_t e0 = r * RUN, e1 = e0 + RUN < nnz ? e0 + RUN : nnz;
        int lo = 0, hi = n;  // the row holding e0: largest v with xadj[v] <= e0
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (xadj[mid] <= e0) lo = mid;
            else hi = mid;
        }
        int v = lo;
        int64_t vend = xadj[v + 1];
        uint64_t m = ~0ull;
        for (int64_t e = e0; e < e1; e++) {
            while (e >= vend) {  // next non-empty row (e < nnz = xadj[n] keeps v < n)
                bfs_lower(key, v, m, ch);
                v++;
                vend = xadj[v + 1];
                m = ~0ull;
            }
            const uint64_t c = key[adj[e]] + 1;  // same root, one hop further
            m = c < m ? c : m;
        }
        bfs_lower(key, v, m, ch);
    }
    if (ch) changed[0] = 1;
}

__global__ __launch_bounds__(CB) void k_bfs_weights(int n, const int32_t *vw, const int32_t *order, int64_t *w)
{
    for (int i = blockIdx.x * CB + threadIdx.x; i < n; i += gridDim.x * CB) w[i] = vw ? vw[order[i]] : 1;
}

// a * b <= c * d for unsigned 64-bit operands (128-bit products)
__device__ __forceinline__ bool mul_le(uint64_t a, uint64_t b, uint64_t c, uint64_t d)
{
    const uint64_t h1 = __umul64hi(a, b), h2 = __umul64hi(c, d);
    return h1 < h2 || (h1 == h2 && a * b <= c * d);
}

// The vertex at position i, with weight b before it, goes to the largest part
// p with p W <= b k, i.e. floor(b k / W) (W = 0: part 0).
__global__ __launch_bounds__(CB) void k_bfs_assign(int n, int k, const int32_t *order, const int64_t *w,
                                                   const int64_t *incl, int32_t *part)
{
    const uint64_t W = (uint64_t)incl[n - 1];
    for (int i = blockIdx.x * CB + threadIdx.x; i < n; i += gridDim.x * CB) {
        const uint64_t b = (uint64_t)(incl[i] - w[i]);
        int lo = 0, hi = W ? k - 1 : 0;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (mul_le((uint64_t)mid, W, b, (uint64_t)k)) lo = mid;
            else hi = mid - 1;
        }
        part[order[i]] = lo;
    }
}

int bfs_start(jet_context *ctx, const jet_csr *g, int k, int32_t *part, hipStream_t s)
{
    const int n = g->n;
    if (n == 0) return JET_OK;
    const size_t nn = (size_t)n;
    uint64_t *key = (uint64_t *)ws_get(ctx, WS_TH_KEY, nn * 16);
    int32_t *val = (int32_t *)ws_get(ctx, WS_TH_VAL, nn * 8);
    int64_t *w = (int64_t *)ws_get(ctx, WS_TH_RUN, nn * 16 + 64);
    if (!key || !val || !w) return JET_ENOMEM;
    uint64_t *key2 = key + nn;
    int32_t *val2 = val + nn;
    int64_t *incl = w + nn;
    int32_t *changed = (int32_t *)(incl + nn);
    size_t sort_bytes = 0, scan_bytes = 0;
    JET_TRY(rocprim::radix_sort_pairs(nullptr, sort_bytes, key, key2, val, val2, nn, 0, 64, s));
    JET_TRY(rocprim::inclusive_scan(nullptr, scan_bytes, w, incl, nn, rocprim::plus<int64_t>(), s));
    void *tmp = ws_get(ctx, WS_TH_TMP, std::max(sort_bytes, scan_bytes) + 256);
    if (!tmp) return JET_ENOMEM;
    int32_t *hch = (int32_t *)((char *)ctx->pinned + 2560);
    const int gv = grid_for(ctx, n, CB, 4);
    const int ge = grid_for(ctx, (g->nnz + 15) / 16, CB);
    k_bfs_init<<<gv, CB, 0, s>>>(n, key, val);
    // after p passes every vertex within p hops of its component's smallest
    // id (along a shortest path) holds its final key, and BFS distances are
    // below n: at most n passes change anything. Chunks of 4 passes, one look
    // each; n / 4 + 2 chunks cover n passes and the pass that finds no change.
    constexpr int CHUNK = 4;
    bool done = false;
    for (int64_t c = 0; c <= nn / CHUNK + 1 && !done; c++) {
        JET_TRY(hipMemsetAsync(changed, 0, 4, s));
        if (g->nnz > 0)
            for (int i = 0; i < CHUNK; i++) k_bfs_relax<<<ge, CB, 0, s>>>(n, g->nnz, g->xadj, g->adjncy, key, changed);
        JET_TRY(hipMemcpyAsync(hch, changed, 4, hipMemcpyDeviceToHost, s));
        JET_TRY(stream_wait(ctx, s));
        done = *hch == 0;
    }
    if (!done) return JET_EGRAPH;  // not reached for any CSR: the bound above holds for every adjacency
    size_t b = sort_bytes;
    JET_TRY(rocprim::radix_sort_pairs(tmp, b, key, key2, val, val2, nn, 0, 64, s));
    k_bfs_weights<<<gv, CB, 0, s>>>(n, g->vwgt, val2, w);
    b = scan_bytes;
    JET_TRY(rocprim::inclusive_scan(tmp, b, w, incl, nn, rocprim::plus<int64_t>(), s));
    k_bfs_assign<<<gv, CB, 0, s>>>(n, k, val2, w, incl, part);
    return hip_status(ctx, hipGetLastError());
}

// The start of the coarsest level: graph-growing with JET_F_BFS_START, else
// the seeded uniform random partition.
int coarsest_start(jet_context *ctx, const jet_csr *g, const jet_params *p, int32_t *part, hipStream_t s)
{
    if (p->flags & JET_F_BFS_START) return bfs_start(ctx, g, p->k, part, s);
    return random_partition(ctx, g->n, p->k, p->seed, part, s);
}

extern "C" int jet_bfs_start(jet_context *ctx, const jet_csr *g, int32_t k, int32_t *part, void *stream)
{
    if (!ctx || !g || (!part && g->n > 0) || k < 1) return JET_EINVAL;
    if (k > KMAX) return JET_ELIMIT;
    hipStream_t s = (hipStream_t)stream;
    JET_TRY(hipSetDevice(ctx->device));
    const int st = check_graph(ctx, g, 0, s);
    if (st) return st;
    return bfs_start(ctx, g, k, part, s);
}

void hierarchy_release(jet_hierarchy *h) { hier_release(h); }

int random_partition(jet_context *ctx, int n, int k, uint64_t seed, int32_t *part, hipStream_t s)
{
    if (n > 0) k_random_part<<<grid_for(ctx, n, CB, 4), CB, 0, s>>>(n, k, mix64(seed ^ 1ULL), part);
    return hip_status(ctx, hipGetLastError());
}

int project_partition(jet_context *ctx, int n, const int32_t *map, const int32_t *coarse, int32_t *fine, hipStream_t s)
{
    if (n > 0) k_project<<<grid_for(ctx, n, CB, 4), CB, 0, s>>>(n, map, coarse, fine);
    return hip_status(ctx, hipGetLastError());
}

}  // namespace jet

using namespace jet;

extern "C" int jet_coarsen(jet_context *ctx, const jet_csr *g, const jet_params *params, jet_hierarchy **out,
                           void *stream)
{
    if (!ctx || !g || !params || !out) return JET_EINVAL;
    *out = nullptr;
    if (params->k < 1) return JET_EINVAL;
    if (params->k > KMAX) return JET_ELIMIT;
    hipStream_t s = (hipStream_t)stream;
    JET_TRY(hipSetDevice(ctx->device));
    int st = check_graph(ctx, g, params->flags, s);
    if (st) return st;
    jet_hierarchy *h = new (std::nothrow) jet_hierarchy();
    if (!h) return JET_ENOMEM;
    JET_TRY(hipEventRecord(ctx->ev[0], s));
    st = build_hierarchy(ctx, g, params, h, s);
    if (st) { hier_release(h); delete h; return st; }
    JET_TRY(hipEventRecord(ctx->ev[1], s));
    JET_TRY(stream_wait(ctx, s));
    (void)hipEventElapsedTime(&h->ms_coarsen, ctx->ev[0], ctx->ev[1]);
    *out = h;
    return JET_OK;
}

extern "C" int jet_hierarchy_levels(const jet_hierarchy *h) { return h ? h->nlevels : 0; }

extern "C" int jet_hierarchy_level(const jet_hierarchy *h, int level, jet_csr *view, const int32_t **map)
{
    if (!h || !view || level < 0 || level >= h->nlevels) return JET_EINVAL;
    *view = h->lv[level];
    if (map) *map = h->maps[level];
    return JET_OK;
}

extern "C" void jet_hierarchy_free(jet_hierarchy *h)
{
    if (!h) return;
    (void)hipSetDevice(h->device);
    hier_release(h);
    delete h;
}

extern "C" int jet_partition(jet_context *ctx, const jet_csr *g, const jet_params *params, int32_t *part_out,
                             jet_stats *stats, jet_trace *trace, void *stream)
{
    if (!ctx || !g || !params || (!part_out && g->n > 0)) return JET_EINVAL;
    if (params->k < 1 || params->lambda_ppm < 0 || (params->flags & JET_F_ASYNC)) return JET_EINVAL;
    if (params->k > KMAX) return JET_ELIMIT;
    hipStream_t s = (hipStream_t)stream;
    JET_TRY(hipSetDevice(ctx->device));
    int st = check_graph(ctx, g, params->flags, s);
    if (st) return st;
    if (trace) { trace->count = 0; trace->total = 0; }
    hipEvent_t e0, e1, e2;
    JET_TRY(hipEventCreate(&e0));
    JET_TRY(hipEventCreate(&e1));
    JET_TRY(hipEventCreate(&e2));
    JET_TRY(hipEventRecord(e0, s));
    // the coarse levels live in the context's arena (kept between calls)
    jet_hierarchy h;
    h.arena = &ctx->part_arena;
    st = build_hierarchy(ctx, g, params, &h, s);
    JET_TRY(hipEventRecord(e1, s));
    int levels = h.nlevels;
    jet_stats agg;
    memset(&agg, 0, sizeof(agg));
    if (st == JET_OK && g->n > 0) {
        // start of the coarsest graph (seeded random or graph-growing), then refine upward
        const int l = levels - 1;
        const int nmax = g->n;
        int32_t *pa = (int32_t *)ws_get(ctx, WS_C10, (size_t)nmax * 4);
        int32_t *pb = (int32_t *)ws_get(ctx, WS_C11, (size_t)nmax * 4);
        if (!pa || !pb) st = JET_ENOMEM;
        if (st == JET_OK) {
            st = coarsest_start(ctx, &h.lv[l], params, pa, s);
        }
        if (st == JET_OK) {
            int32_t *cur = pa, *other = pb;
            int64_t cut_prev = -1;  // cut of the coarser level's result, which the projection keeps
            for (int i = l; i >= 0 && st == JET_OK; i--) {
                if (i < l) {
                    int32_t *dst = i == 0 ? part_out : other;
                    k_project<<<grid_for(ctx, h.lv[i].n, CB, 4), CB, 0, s>>>(h.lv[i].n, h.maps[i], cur, dst);
                    other = cur;
                    cur = dst;
                } else if (i == 0) {
                    JET_TRY(hipMemcpyAsync(part_out, cur, sizeof(int32_t) * g->n, hipMemcpyDeviceToDevice, s));
                    cur = part_out;
                }
                jet_params q = *params;
                q.level = i;
                q.flags &= ~(uint32_t)JET_F_VALIDATE;
                if (i > 0) q.flags &= ~(uint32_t)JET_F_PROFILE;  // only the finest level is profiled
                jet_stats ls;
                int32_t cnt = 0, tot = 0;
                jet_trace_rec *recs = nullptr;
                int32_t cap = 0;
                if (trace && trace->recs && trace->count < trace->cap) {
                    recs = trace->recs + trace->count;
                    cap = trace->cap - trace->count;
                }
                st = refine_level(ctx, &h.lv[i], &q, cur, nullptr, &ls, recs, cap, &cnt, &tot, s,
                                  i < l ? cut_prev : -1);
                if (st) break;
                cut_prev = ls.cut;
                if (trace) { trace->count += cnt; trace->total += tot; }
                agg.iters += ls.iters;
                agg.lp_iters += ls.lp_iters;
                agg.rw_iters += ls.rw_iters;
                agg.rs_iters += ls.rs_iters;
                agg.ms_refine += ls.ms_refine;
                agg.ms_init += ls.ms_init;
                if (i == 0) {
                    agg.ms_gain = ls.ms_gain;
                    agg.gain_passes = ls.gain_passes;
                    agg.gain_entries = ls.gain_entries;
                    agg.gain_rows = ls.gain_rows;
                    agg.gain_vertices = ls.gain_vertices;
                    agg.cut = ls.cut;
                    agg.max_part_weight = ls.max_part_weight;
                    agg.o = ls.o;
                    agg.sigma = ls.sigma;
                    agg.total_weight = ls.total_weight;
                    agg.balanced = ls.balanced;
                }
            }
        }
    }
    if (st == JET_OK) {
        JET_TRY(hipEventRecord(e2, s));
        JET_TRY(stream_wait(ctx, s));
    }
    float ms_c = 0, ms_t = 0;
    if (st == JET_OK) {
        (void)hipEventElapsedTime(&ms_c, e0, e1);
        (void)hipEventElapsedTime(&ms_t, e0, e2);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(e2);
    if (st) (void)hipStreamSynchronize(s);  // nothing queued may still use the arena
    hier_release(&h);
    if (st) return st;
    if (stats) {
        *stats = agg;
        stats->levels = levels;
        stats->ms_coarsen = ms_c;
        stats->ms_total = ms_t;
    }
    return JET_OK;
}
