// Jet refinement on gfx950: Jetlp with the afterburner (Algorithm 4), weak and
// strong rebalancing (Algorithm 5 and the strong variant of Section 4.2.2),
// synchronous move application, and the refinement loop of Algorithm 3 run by
// a device-side controller.
//
// Design (one MI355X):
//  * Connectivity conn(v, .) is rebuilt per pass in LDS. Vertices are binned
//    by degree: <= 32 -> 8-lane groups (32 groups per 256-thread block),
//    <= 1024 -> one wave, larger -> one block. Each group owns a dense int32
//    table of k entries; neighbours add their edge weight with LDS atomics,
//    then read-and-clear the entry of their own part with an atomic exchange,
//    so every adjacent part is seen exactly once and the table is left zero.
//    Integer sums are exact in any order; argmax ties break by part id, so the
//    result does not depend on scheduling.
//  * Per-vertex Jetlp state is one 8-byte record (P_s, P_d + in-X flag, F), so
//    the afterburner's neighbour gather is a single load.
//  * Rebalancing orders evictions by (loss slot, vertex id): a per-(part, slot)
//    weight histogram fixes the cut-off slot of every oversized part; inside
//    that slot, vertex-ordered prefix sums per part come from per-tile sums,
//    a per-part scan over tiles, and a wave-level ballot/scan inside each tile.
//  * A single-block controller kernel decides each iteration's kind from
//    device state; every other kernel exits at once when its kind is not
//    selected, so iterations are enqueued in chunks with one host sync each.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "jet_device.h"
#include "jet_internal.h"

namespace jet {

// ------------------------------------------------------------------ set-up --

// Copies P_0, clears per-vertex state, sums vertex and part weights, counts
// degree classes and checks part ids / vertex weights / xadj monotonicity.
__global__ __launch_bounds__(BLOCK) void k_init_vertices(KArgs a, const int32_t *part_in)
{
    extern __shared__ int32_t s_w[];  // [k] block-partial part weights
    __shared__ int64_t s_red[BLOCK / 64];
    __shared__ uint64_t s_redu[BLOCK / 64];
    __shared__ int32_t s_cls[NCLS];
    for (int p = threadIdx.x; p < a.k; p += BLOCK) s_w[p] = 0;
    if (threadIdx.x < NCLS) s_cls[threadIdx.x] = 0;
    __syncthreads();
    int64_t wsum = 0;
    uint64_t dig = 0;
    int bad_part = 0, bad_graph = 0;
    const int stride = gridDim.x * BLOCK;
    for (int v = blockIdx.x * BLOCK + threadIdx.x; v < a.n; v += stride) {
        int p = part_in[v];
        if (p < 0 || p >= a.k) { bad_part = 1; p = 0; }
        a.P[v] = p;
        a.dest[v] = -1;
        a.lock[v] = -1;
        int vwv = a.vw ? a.vw[v] : 1;
        if (vwv < 1) bad_graph = 1;
        int64_t d = a.xadj[v + 1] - a.xadj[v];
        if (d < 0) { bad_graph = 1; d = 0; }
        int c = d == 0 ? CLS_Z : (d <= S_MAXDEG ? CLS_S : (d <= M_MAXDEG ? CLS_M : CLS_L));
        atomicAdd(&s_cls[c], 1);
        atomicAdd(&s_w[p], vwv);
        wsum += vwv;
        dig += mix64(((uint64_t)(uint32_t)v << 32) | (uint32_t)p);
    }
    wsum = block_sum<BLOCK>(wsum, s_red);
    dig = block_sum<BLOCK>(dig, s_redu);
    if (bad_part) a.ctl->bad_part = 1;
    if (bad_graph) a.ctl->bad_graph = 1;
    if (threadIdx.x == 0) {
        atomicAdd((unsigned long long *)&a.ctl->wsum, (unsigned long long)wsum);
        atomicAdd((unsigned long long *)&a.ctl->digest, (unsigned long long)dig);
    }
    if (threadIdx.x < NCLS && s_cls[threadIdx.x]) atomicAdd(&a.ctl->bincnt[threadIdx.x], s_cls[threadIdx.x]);
    for (int p = threadIdx.x; p < a.k; p += BLOCK)
        if (s_w[p]) atomicAdd((unsigned long long *)&a.w[p], (unsigned long long)(int64_t)s_w[p]);
}

// Edge pass: cut of P_0, total edge weight, neighbour-range / self-loop /
// weight checks. Each thread walks a run of 16 consecutive CSR entries.
__global__ __launch_bounds__(BLOCK) void k_init_edges(KArgs a, int64_t nnz)
{
    __shared__ int64_t s_red[BLOCK / 64];
    constexpr int RUN = 16;
    int64_t cut = 0, ews = 0;
    int bad = 0;
    const int64_t nruns = (nnz + RUN - 1) / RUN;
    for (int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x; r < nruns; r += (int64_t)gridDim.x * BLOCK) {
        int64_t e0 = r * RUN, e1 = e0 + RUN < nnz ? e0 + RUN : nnz;
        // row containing e0: last v with xadj[v] <= e0
        int lo = 0, hi = a.n;  // invariant xadj[lo] <= e0 < xadj[hi] (xadj[n] = nnz > e0)
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (a.xadj[mid] <= e0) lo = mid; else hi = mid;
        }
        int v = lo;
        int64_t vend = a.xadj[v + 1];
        int pv = a.P[v];
        for (int64_t e = e0; e < e1; e++) {
            while (e >= vend && v < a.n - 1) { v++; vend = a.xadj[v + 1]; pv = a.P[v]; }
            int u = a.adj[e];
            int wt = a.ew ? a.ew[e] : 1;
            if (u < 0 || u >= a.n || u == v || wt < 1) { bad = 1; continue; }
            ews += wt;
            if (u > v && a.P[u] != pv) cut += wt;
        }
    }
    cut = block_sum<BLOCK>(cut, s_red);
    ews = block_sum<BLOCK>(ews, s_red);
    if (bad) a.ctl->bad_graph = 1;
    if (threadIdx.x == 0) {
        atomicAdd((unsigned long long *)&a.ctl->cut, (unsigned long long)cut);
        atomicAdd((unsigned long long *)&a.ctl->ewsum, (unsigned long long)ews);
    }
}

// Fill the degree-class vertex lists.
__global__ __launch_bounds__(BLOCK) void k_fill_bins(KArgs a, int32_t *bins, int32_t *fill)
{
    const int stride = gridDim.x * BLOCK;
    const int nloop = (a.n + stride - 1) / stride;
    for (int it = 0; it < nloop; it++) {
        int v = it * stride + blockIdx.x * BLOCK + threadIdx.x;
        bool ok = v < a.n;
        int c = -1;
        if (ok) {
            int64_t d = a.xadj[v + 1] - a.xadj[v];
            c = d == 0 ? CLS_Z : (d <= S_MAXDEG ? CLS_S : (d <= M_MAXDEG ? CLS_M : CLS_L));
        }
#pragma unroll
        for (int cc = 0; cc < NCLS; cc++) wave_append(c == cc, &fill[cc], bins + a.binoff[cc], v);
    }
}

// -------------------------------------------------------------- controller --

// Oversized parts A = {w > o}, valid destinations B = {w <= sigma} listed in
// ascending id, and a cleared (part, slot) histogram. Whole block calls.
__device__ void rb_prepare(const KArgs &a)
{
    __shared__ int32_t s_scan[BLOCK / 64];
    Ctl *c = a.ctl;
    const int64_t o = c->o, sigma = c->sigma;
    int32_t carry = 0, nA = 0;
    for (int base = 0; base < a.k; base += BLOCK) {
        int p = base + threadIdx.x;
        int inA = 0, inB = 0;
        if (p < a.k) {
            int64_t wp = a.w[p];
            inA = wp > o;
            inB = wp <= sigma;
            a.isA[p] = (uint8_t)inA;
            a.isB[p] = (uint8_t)inB;
        }
        int32_t tot;
        int32_t pos = block_excl_scan<BLOCK>((int32_t)inB, s_scan, tot);
        if (inB) a.Blist[carry + pos] = p;
        carry += tot;
        int32_t ta;
        block_excl_scan<BLOCK>((int32_t)inA, s_scan, ta);
        nA += ta;
    }
    for (int i = threadIdx.x; i < a.k * NSLOT; i += BLOCK) a.hist[i] = 0;
    if (threadIdx.x == 0) { c->nB = carry; c->nA = nA; }
}

__device__ __forceinline__ void clear_accumulators(Ctl *c)
{
    c->nX = 0; c->nM = 0;
    c->dcut = 0; c->moved_w = 0; c->ddigest = 0;
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
        if (cc.balanced) { kind = KIND_LP; cc.lp_id++; cc.wcount = 0; cc.n_lp++; }
        else if (cc.wcount < cc.bmax) { kind = KIND_RW; cc.wcount++; cc.n_rw++; }
        else { kind = KIND_RS; cc.wcount++; cc.n_rs++; }
    }
    cc.kind = kind;
    clear_accumulators(&cc);
    return kind;
}

// Whole-block part of starting an iteration: clear the counter shards and,
// for rebalancing, build A, B and clear the histogram.
__device__ __forceinline__ void begin_iteration(const KArgs &a, int kind)
{
    for (int i = threadIdx.x; i < NSTAT * NSHARD; i += blockDim.x) a.bstat[i] = 0;
    if (kind == KIND_RW || kind == KIND_RS) rb_prepare(a);
}

// Derived loop state after the set-up passes.
__global__ __launch_bounds__(BLOCK) void k_ctl_setup(KArgs a, int64_t W, int64_t o, int64_t sigma)
{
    __shared__ uint64_t s_red[BLOCK / 64];
    Ctl *c = a.ctl;
    uint64_t m = 0;
    for (int p = threadIdx.x; p < a.k; p += BLOCK) {
        uint64_t x = (uint64_t)a.w[p];
        m = x > m ? x : m;
        a.wbest[p] = a.w[p];
    }
    m = block_max_u64<BLOCK>(m, s_red);
    __shared__ int s_next;
    if (threadIdx.x == 0) {
        Ctl cc = *c;
        cc.W = W; cc.o = o; cc.sigma = sigma;
        cc.maxw = (int64_t)m;
        cc.balanced = (int64_t)m <= o;
        cc.bal_best = cc.balanced;
        cc.cut_best = cc.cut;
        cc.maxw_best = cc.maxw;
        s_next = ctl_next(cc);  // iteration 0
        *c = cc;
    }
    __syncthreads();
    begin_iteration(a, s_next);
}

// Adds a block's partial counter into one of NSHARD shards of its stat row
// (shards spread the atomics; the controller sums NSHARD values per row).
__device__ __forceinline__ void shard_add(const KArgs &a, int row, int64_t val)
{
    if (val) atomicAdd((unsigned long long *)&a.bstat[row * NSHARD + (blockIdx.x & (NSHARD - 1))],
                       (unsigned long long)val);
}

// Single-step entry points: force one iteration of `kind` at index t. For
// Jetlp, lock flags become stamps of the previous Jetlp (id 0).
__global__ __launch_bounds__(BLOCK) void k_force_step(KArgs a, int kind, int t, const uint8_t *locked)
{
    Ctl *c = a.ctl;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c->kind = kind;
        c->t = t;
        c->lp_id = 1;
        clear_accumulators(c);
    }
    if (locked)
        for (int v = blockIdx.x * BLOCK + threadIdx.x; v < a.n; v += gridDim.x * BLOCK) a.lock[v] = locked[v] ? 0 : -1;
    if (blockIdx.x == 0) {
        __syncthreads();
        begin_iteration(a, kind);
    }
}

// Defaults of the step outputs for vertices no row kernel visits (isolated).
__global__ __launch_bounds__(BLOCK) void k_step_defaults(KArgs a, const int32_t *part)
{
    for (int v = blockIdx.x * BLOCK + threadIdx.x; v < a.n; v += gridDim.x * BLOCK) {
        if (a.dbg_F) { a.dbg_F[v] = INT64_MIN; a.dbg_cs[v] = 0; a.dbg_F2[v] = 0; a.dbg_pd[v] = part[v]; }
        if (a.dbg_loss) { a.dbg_loss[v] = INT64_MIN; a.dbg_slot[v] = -1; }
    }
}

__global__ __launch_bounds__(BLOCK) void k_lp_outputs(KArgs a, uint8_t *inX, uint8_t *move)
{
    for (int v = blockIdx.x * BLOCK + threadIdx.x; v < a.n; v += gridDim.x * BLOCK) {
        const bool iso = a.xadj[v + 1] == a.xadj[v];
        inX[v] = iso ? 0 : (uint8_t)((a.rec[v].x & 0xFFFF) != 0);
        move[v] = a.dest[v] >= 0;
    }
}

constexpr int CTL_NT = BLOCK;  // threads of the end-of-iteration controller

__global__ __launch_bounds__(CTL_NT) void k_ctl_end(KArgs a)
{
    __shared__ uint64_t s_red[CTL_NT / 64];
    __shared__ int64_t s_red64[CTL_NT / 64];
    __shared__ int s_improved, s_next;
    Ctl *c = a.ctl;
    const int kind = c->kind;
    if (kind == KIND_DONE) return;
    uint64_t m = 0;
    for (int p = threadIdx.x; p < a.k; p += CTL_NT) {
        uint64_t x = (uint64_t)a.w[p];
        m = x > m ? x : m;
    }
    m = block_max_u64<CTL_NT>(m, s_red);
    // this iteration's counters (NSHARD shards per row)
    int64_t px = 0, pm = 0, pdc = 0, pmw = 0;
    uint64_t pdg = 0;
    int64_t pe = 0, pr = 0, pv = 0;
    if (threadIdx.x < NSHARD) {
        const int i = threadIdx.x;
        px = a.bstat[ST_X * NSHARD + i];
        pm = a.bstat[ST_M * NSHARD + i];
        pdc = a.bstat[ST_DCUT * NSHARD + i];
        pmw = a.bstat[ST_MW * NSHARD + i];
        pdg = (uint64_t)a.bstat[ST_DIG * NSHARD + i];
        if (kind == KIND_LP) {
            pe = a.bstat[ST_E * NSHARD + i];
            pr = a.bstat[ST_R * NSHARD + i];
            pv = a.bstat[ST_V * NSHARD + i];
        }
    }
    pe = block_sum<CTL_NT>(pe, s_red64);
    pr = block_sum<CTL_NT>(pr, s_red64);
    pv = block_sum<CTL_NT>(pv, s_red64);
    px = block_sum<CTL_NT>(px, s_red64);
    pm = block_sum<CTL_NT>(pm, s_red64);
    pdc = block_sum<CTL_NT>(pdc, s_red64);
    pmw = block_sum<CTL_NT>(pmw, s_red64);
    pdg = block_sum<CTL_NT>(pdg, s_red);
    if (threadIdx.x == 0) {
        // one load of the whole state, one store: no dependent global round trips
        Ctl cc = *c;
        const int64_t maxw = (int64_t)m;
        const int nM = (int)pm, nXl = (int)px;
        cc.nX = nXl; cc.nM = nM;
        cc.dcut = pdc; cc.moved_w = pmw; cc.ddigest = pdg;
        cc.prof_e += pe; cc.prof_r += pr; cc.prof_v += pv;
        cc.cut += cc.dcut;
        cc.digest += cc.ddigest;
        cc.maxw = maxw;
        const int bal = maxw <= cc.o;
        cc.balanced = bal;
        int improved = 0;
        if (bal) {
            if (!cc.bal_best) {
                // a balanced partition always replaces an imbalanced best
                improved = 1; cc.bal_best = 1; cc.cut_best = cc.cut; cc.maxw_best = maxw; cc.stall = 0;
            } else if (cc.cut < cc.cut_best) {
                // only a gain beyond the tolerance phi restarts the count
                if ((int64_t)cc.phi_den * cc.cut < (int64_t)cc.phi_num * cc.cut_best) cc.stall = 0;
                improved = 1; cc.cut_best = cc.cut; cc.maxw_best = maxw;
            }
        } else if (!cc.bal_best && maxw < cc.maxw_best) {
            improved = 1; cc.maxw_best = maxw; cc.cut_best = cc.cut; cc.stall = 0;
        }
        cc.copy_best = improved;
        if (a.kinds && cc.t < KIND_LOG) a.kinds[cc.t] = (int8_t)kind;
        if (a.trace && cc.t < cc.trace_cap) {
            jet_trace_rec r;
            r.level = cc.level; r.t = cc.t; r.kind = kind;
            r.nX = nXl;
            r.nM = nM; r.stall = cc.stall; r.wcount = cc.wcount; r.balanced = bal;
            r.moved_w = cc.moved_w; r.cut = cc.cut; r.maxw = maxw; r.best_cut = cc.cut_best;
            r.digest = cc.digest;
            a.trace[cc.t] = r;
        }
        cc.t++;
        s_next = ctl_next(cc);
        *c = cc;
        s_improved = improved;
    }
    __syncthreads();
    if (s_improved)
        for (int p = threadIdx.x; p < a.k; p += CTL_NT) a.wbest[p] = a.w[p];
    begin_iteration(a, s_next);
}

__global__ __launch_bounds__(BLOCK) void k_copy_best(KArgs a)
{
    if (!a.ctl->copy_best) return;
    const int stride = gridDim.x * BLOCK;
    if ((((uintptr_t)a.best | (uintptr_t)a.P) & 15) == 0) {
        const int n4 = a.n >> 2;
        const int4 *src = (const int4 *)a.P;
        int4 *dst = (int4 *)a.best;
        for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n4; i += stride) dst[i] = src[i];
        for (int v = (n4 << 2) + blockIdx.x * BLOCK + threadIdx.x; v < a.n; v += stride) a.best[v] = a.P[v];
    } else {
        for (int v = blockIdx.x * BLOCK + threadIdx.x; v < a.n; v += stride) a.best[v] = a.P[v];
    }
}

// ------------------------------------------------------ connectivity core --

// Group of G lanes gathers the neighbours of v (deg <= G*R) into table `tab`
// and reads every adjacent part's total back exactly once: on return pu[r] is
// the part of neighbour slot r (-1 if none) and cu[r] its connectivity for the
// first lane that claimed it, else 0. The table is left all-zero.
template <int G, int R>
__device__ __forceinline__ void group_conn_row(const KArgs &a, int64_t s, int deg, int gl, int32_t *tab, int (&pu)[R],
                                               int (&cu)[R])
{
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int idx = gl + r * G;
        pu[r] = -1;
        if (idx < deg) {
            const int u = a.adj[s + idx];
            const int wt = a.ew ? a.ew[s + idx] : 1;
            pu[r] = a.P[u];
            atomicAdd(&tab[pu[r]], wt);
        }
    }
    lds_fence_wave();
#pragma unroll
    for (int r = 0; r < R; r++) cu[r] = pu[r] >= 0 ? atomicExch(&tab[pu[r]], 0) : 0;
    lds_fence_wave();
}

template <int G, int R>
__device__ __forceinline__ void group_conn(const KArgs &a, int v, int gl, int32_t *tab, int (&pu)[R], int (&cu)[R])
{
    const int64_t s = a.xadj[v];
    group_conn_row<G, R>(a, s, (int)(a.xadj[v + 1] - s), gl, tab, pu, cu);
}

// Wave-batched driver of the 8-lane role. Lanes first inspect 64 list
// entries at once (coalesced loads of the id, row offsets and per-vertex
// state); the entries that need row work are queued in LDS and handed to the
// wave's eight 8-lane groups, eight at a time. Metadata round trips are paid
// once per 64 vertices instead of once per vertex, and skipped vertices cost
// no group time.
struct Meta {
    int v, ps, deg, aux;
    int64_t s;
};

template <int G, class Pre, class Row>
__device__ __forceinline__ void wave_batched(const int32_t *list, int cnt, int32_t *q, int wid, int nwaves, Pre pre,
                                             Row row)
{
    const int lane = threadIdx.x & 63, g = lane / G, gl = lane & (G - 1);
    for (int base = wid * 64; base < cnt; base += nwaves * 64) {
        const int i = base + lane;
        Meta m{0, 0, 0, 0, 0};
        bool act = false;
        if (i < cnt) {
            m.v = list[i];
            act = pre(m);
        }
        const uint64_t mask = __ballot(act);
        if (act) q[__popcll(mask & ((1ull << lane) - 1ull))] = lane;
        lds_fence_wave();
        const int nact = __popcll(mask);
        for (int sb = 0; sb < nact; sb += 64 / G) {
            const int slot = sb + g;
            const bool has = slot < nact;
            const int src = q[has ? slot : 0];
            Meta t;
            t.v = __shfl(m.v, src, 64);
            t.ps = __shfl(m.ps, src, 64);
            t.deg = __shfl(m.deg, src, 64);
            t.aux = __shfl(m.aux, src, 64);
            t.s = __shfl(m.s, src, 64);
            if (has) row(t, gl);
        }
        lds_fence_wave();
    }
}

template <class Pre, class Row>
__device__ __forceinline__ void wave_batched8(const int32_t *list, int cnt, int32_t *q, int wid, int nwaves, Pre pre,
                                              Row row)
{
    wave_batched<8>(list, cnt, q, wid, nwaves, pre, row);
}

// Whole block gathers the neighbours of v into `tab` (k entries).
__device__ __forceinline__ void block_fill(const KArgs &a, int v, int32_t *tab)
{
    const int64_t s = a.xadj[v], e = a.xadj[v + 1];
    for (int64_t i = s + threadIdx.x; i < e; i += BLOCK) {
        const int u = a.adj[i];
        atomicAdd(&tab[a.P[u]], a.ew ? a.ew[i] : 1);
    }
    __syncthreads();
}

// Largest-connectivity key: connectivity in the high word, ~part in the low
// word, so ties go to the smaller part id.
__device__ __forceinline__ uint64_t conn_key(int c, int p)
{
    return ((uint64_t)(uint32_t)c << 32) | (uint32_t)(~p);
}

// -------------------------------------------------------------- Jetlp gain --

// Writes rec[v] and appends v to its class's X list when it passes the
// first filter (eq. gainconn_filter).
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
    a.rec[v] = r;
    if (a.dbg_F) {
        a.dbg_F[v] = F;
        a.dbg_cs[v] = cs;
        a.dbg_pd[v] = pd;
    }
    return inx;
}

__device__ __forceinline__ void gain_locked(const KArgs &a, int v, int ps)
{
    a.rec[v] = make_int2(ps << 16, 0);
    if (a.dbg_F) { a.dbg_F[v] = INT64_MIN; a.dbg_cs[v] = 0; a.dbg_pd[v] = ps; }
}

struct GainCount {
    int nx = 0;
    int64_t e = 0, r = 0, v = 0;
};

template <int G, int R>
__device__ void gain_groups(const KArgs &a, int cls, int32_t *tab, int gid, int ngroups, int lp_prev, int cn, int cd,
                            GainCount &gc)
{
    const int gl = threadIdx.x & (G - 1);
    const int32_t *list = a.bins + a.binoff[cls];
    const int cnt = a.binoff[cls + 1] - a.binoff[cls];
    for (int i = gid; i < cnt; i += ngroups) {
        const int v = list[i];
        const int ps = a.P[v];
        if (gl == 0) gc.v++;
        if (a.lock[v] == lp_prev) {
            if (gl == 0) gain_locked(a, v, ps);
            continue;
        }
        if (gl == 0) { gc.r++; gc.e += a.xadj[v + 1] - a.xadj[v]; }
        int pu[R], cu[R];
        group_conn<G, R>(a, v, gl, tab, pu, cu);
        uint64_t best = 0;
        int cs = 0;
#pragma unroll
        for (int r = 0; r < R; r++) {
            if (cu[r] > 0) {
                if (pu[r] == ps) cs += cu[r];
                else { uint64_t k2 = conn_key(cu[r], pu[r]); best = k2 > best ? k2 : best; }
            }
        }
        best = gmax_u64<G>(best);
        cs = gsum<G>(cs);
        if (gl == 0) gc.nx += gain_finish(a, v, ps, best, cs, cn, cd);
    }
}

__device__ void gain_blocks(const KArgs &a, int cls, int32_t *tab, int bid, int nblocks, int lp_prev, int cn, int cd,
                            GainCount &gc)
{
    __shared__ uint64_t s_red[BLOCK / 64];
    __shared__ int32_t s_red32[BLOCK / 64];
    const int32_t *list = a.bins + a.binoff[cls];
    const int cnt = a.binoff[cls + 1] - a.binoff[cls];
    for (int i = bid; i < cnt; i += nblocks) {
        const int v = list[i];
        const int ps = a.P[v];
        if (threadIdx.x == 0) gc.v++;
        if (a.lock[v] == lp_prev) {
            if (threadIdx.x == 0) gain_locked(a, v, ps);
            continue;
        }
        if (threadIdx.x == 0) { gc.r++; gc.e += a.xadj[v + 1] - a.xadj[v]; }
        block_fill(a, v, tab);
        uint64_t best = 0;
        int cs = 0;
        for (int p = threadIdx.x; p < a.k; p += BLOCK) {
            const int c = tab[p];
            if (c) {
                tab[p] = 0;
                if (p == ps) cs = c;
                else { uint64_t k2 = conn_key(c, p); best = k2 > best ? k2 : best; }
            }
        }
        best = block_max_u64<BLOCK>(best, s_red);
        cs = block_sum<BLOCK>(cs, s_red32);
        if (threadIdx.x == 0) gc.nx += gain_finish(a, v, ps, best, cs, cn, cd);
    }
}

// Role layout of the LDS-table kernels: blocks [0, gS) serve the classes
// mapped to the 8-lane role, the next gM blocks the wave role, the next gL
// blocks the block role, and (rebalancing only) the last gZ blocks isolated
// vertices.
// One kernel per role (8-lane groups, waves, blocks), so each keeps its own
// register budget. Group tables are padded to k + 1 ints so the tables of
// neighbouring groups start in different LDS banks. Block partials of |X|
// land at offset `boff` of the counter row.
template <int ROLE, int GS = 8>
__global__ __launch_bounds__(BLOCK) void k_gain(KArgs a, int nblk, int boff)
{
    if (a.ctl->kind != KIND_LP) return;
    extern __shared__ int32_t lds[];
    __shared__ int32_t s_red32[BLOCK / 64];
    const int lp_prev = a.ctl->lp_id - 1;
    const int cn = a.ctl->c_num, cd = a.ctl->c_den;
    const int stride = a.k + 1;
    GainCount gc;
    if (ROLE == 1) {
        constexpr int RS_ = 32 / GS;
        const int ng = BLOCK / GS;
        for (int i = threadIdx.x; i < ng * stride; i += BLOCK) lds[i] = 0;
        __syncthreads();
        int32_t *tab = lds + (threadIdx.x / GS) * stride;
        int32_t *q = lds + ng * stride + (threadIdx.x >> 6) * 64;
        const int wid = blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6), nwaves = nblk * (BLOCK / 64);
        for (int c = 1; c < NCLS; c++) {
            if (a.tmap[c] != 1) continue;
            wave_batched<GS>(
                a.bins + a.binoff[c], a.binoff[c + 1] - a.binoff[c], q, wid, nwaves,
                [&](Meta &m) -> bool {
                    m.ps = a.P[m.v];
                    gc.v++;
                    if (a.lock[m.v] == lp_prev) {
                        gain_locked(a, m.v, m.ps);
                        return false;
                    }
                    m.s = a.xadj[m.v];
                    m.deg = (int)(a.xadj[m.v + 1] - m.s);
                    gc.r++;
                    gc.e += m.deg;
                    return true;
                },
                [&](const Meta &t, int gl) {
                    int pu[RS_], cu[RS_];
                    group_conn_row<GS, RS_>(a, t.s, t.deg, gl, tab, pu, cu);
                    uint64_t best = 0;
                    int cs = 0;
#pragma unroll
                    for (int r = 0; r < RS_; r++) {
                        if (cu[r] > 0) {
                            if (pu[r] == t.ps) cs += cu[r];
                            else { uint64_t k2 = conn_key(cu[r], pu[r]); best = k2 > best ? k2 : best; }
                        }
                    }
                    best = gmax_u64<GS>(best);
                    cs = gsum<GS>(cs);
                    if (gl == 0) gc.nx += gain_finish(a, t.v, t.ps, best, cs, cn, cd);
                });
        }
    } else if (ROLE == 2) {
        const int ng = BLOCK / 64;
        for (int i = threadIdx.x; i < ng * stride; i += BLOCK) lds[i] = 0;
        __syncthreads();
        int32_t *tab = lds + (threadIdx.x >> 6) * stride;
        for (int c = 1; c < NCLS; c++)
            if (a.tmap[c] == 2)
                gain_groups<64, 16>(a, c, tab, blockIdx.x * ng + (threadIdx.x >> 6), nblk * ng, lp_prev, cn, cd, gc);
    } else {
        for (int i = threadIdx.x; i < a.k; i += BLOCK) lds[i] = 0;
        __syncthreads();
        for (int c = 1; c < NCLS; c++)
            if (a.tmap[c] == 3) gain_blocks(a, c, lds, blockIdx.x, nblk, lp_prev, cn, cd, gc);
    }
    __shared__ int64_t s_red64[BLOCK / 64];
    const int nx = block_sum<BLOCK>(gc.nx, s_red32);
    const int64_t e = block_sum<BLOCK>(gc.e, s_red64);
    const int64_t r = block_sum<BLOCK>(gc.r, s_red64);
    const int64_t v = block_sum<BLOCK>(gc.v, s_red64);
    if (threadIdx.x == 0) {
        shard_add(a, ST_X, nx);
        shard_add(a, ST_E, e);
        shard_add(a, ST_R, r);
        shard_add(a, ST_V, v);
    }
}

// -------------------------------------------------------------- afterburner --

// F2(v) = sum over neighbours u of w * ([q_u = P_d(v)] - [q_u = P_s(v)]) with
// q_u = P_d(u) when u is in X and precedes v (larger F, or equal F and smaller
// id), else P_s(u). Moves with F2 >= 0 form M.
__device__ __forceinline__ int after_sum_row(const KArgs &a, int v, int64_t s, int deg, int ps, int pd, int Fv, int gl,
                                             int stride)
{
    int sum = 0;
    for (int idx = gl; idx < deg; idx += stride) {
        const int u = a.adj[s + idx];
        const int wt = a.ew ? a.ew[s + idx] : 1;
        const int2 ru = a.rec[u];
        int q = ru.x >> 16;
        const int pdu = (ru.x & 0xFFFF) - 1;
        if (pdu >= 0 && (ru.y > Fv || (ru.y == Fv && u < v))) q = pdu;
        sum += q == pd ? wt : (q == ps ? -wt : 0);
    }
    return sum;
}

template <int G>
__device__ __forceinline__ int after_sum(const KArgs &a, int v, int ps, int pd, int Fv, int gl, int stride)
{
    const int64_t s = a.xadj[v];
    return after_sum_row(a, v, s, (int)(a.xadj[v + 1] - s), ps, pd, Fv, gl, stride);
}

template <int G>
__device__ void after_groups(const KArgs &a, int cls, int gid, int ngroups)
{
    const int gl = threadIdx.x & (G - 1);
    const int32_t *list = a.bins + a.binoff[cls];
    const int cnt = a.binoff[cls + 1] - a.binoff[cls];
    for (int i = gid; i < cnt; i += ngroups) {
        const int v = list[i];
        const int2 r = a.rec[v];
        if ((r.x & 0xFFFF) == 0) continue;  // not in X
        const int ps = r.x >> 16, pd = (r.x & 0xFFFF) - 1;
        int sum = after_sum<G>(a, v, ps, pd, r.y, gl, G);
        sum = gsum<G>(sum);
        if (gl == 0) {
            if (a.dbg_F2) a.dbg_F2[v] = sum;
            if (sum >= 0) a.dest[v] = pd;
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_afterburner(KArgs a)
{
    __shared__ int32_t s_red[BLOCK / 64];
    __shared__ int32_t s_q[BLOCK];
    if (a.ctl->kind != KIND_LP) return;
    int b = blockIdx.x;
    if (b < a.gS) {
        int32_t *q = s_q + (threadIdx.x >> 6) * 64;
        wave_batched8(
            a.bins + a.binoff[CLS_S], a.binoff[CLS_S + 1] - a.binoff[CLS_S], q, b * (BLOCK / 64) + (threadIdx.x >> 6),
            a.gS * (BLOCK / 64),
            [&](Meta &m) -> bool {
                const int2 r = a.rec[m.v];
                if ((r.x & 0xFFFF) == 0) return false;  // not in X
                m.ps = r.x;
                m.aux = r.y;
                m.s = a.xadj[m.v];
                m.deg = (int)(a.xadj[m.v + 1] - m.s);
                return true;
            },
            [&](const Meta &t, int gl) {
                const int ps = t.ps >> 16, pd = (t.ps & 0xFFFF) - 1;
                int sum = after_sum_row(a, t.v, t.s, t.deg, ps, pd, t.aux, gl, 8);
                sum = gsum<8>(sum);
                if (gl == 0) {
                    if (a.dbg_F2) a.dbg_F2[t.v] = sum;
                    if (sum >= 0) a.dest[t.v] = pd;
                }
            });
        return;
    }
    b -= a.gS;
    if (b < a.gM) { after_groups<64>(a, CLS_M, b * (BLOCK / 64) + (threadIdx.x >> 6), a.gM * (BLOCK / 64)); return; }
    b -= a.gM;
    if (b >= a.gL) return;
    const int32_t *list = a.bins + a.binoff[CLS_L];
    const int cnt = a.binoff[CLS_L + 1] - a.binoff[CLS_L];
    for (int i = b; i < cnt; i += a.gL) {
        const int v = list[i];
        const int2 r = a.rec[v];
        if ((r.x & 0xFFFF) == 0) continue;
        const int ps = r.x >> 16, pd = (r.x & 0xFFFF) - 1;
        int sum = after_sum<BLOCK>(a, v, ps, pd, r.y, threadIdx.x, BLOCK);
        sum = block_sum<BLOCK>(sum, s_red);
        if (threadIdx.x == 0) {
            if (a.dbg_F2) a.dbg_F2[v] = sum;
            if (sum >= 0) a.dest[v] = pd;
        }
    }
}

// ------------------------------------------------- cut change of the moves --

// Delta of the cut over the edges of moved vertices: an edge whose two ends
// both move is counted from its smaller end. Also moved weight and digest.
__device__ __forceinline__ int dcut_sum_row(const KArgs &a, int v, int64_t s, int deg, int ps, int pn, int gl,
                                            int stride)
{
    int delta = 0;
    for (int idx = gl; idx < deg; idx += stride) {
        const int u = a.adj[s + idx];
        const int du = a.dest[u];
        if (du >= 0 && u < v) continue;
        const int wt = a.ew ? a.ew[s + idx] : 1;
        const int pu = a.P[u];
        const int pun = du >= 0 ? du : pu;
        delta += wt * ((int)(pn != pun) - (int)(ps != pu));
    }
    return delta;
}

__device__ __forceinline__ int dcut_sum(const KArgs &a, int v, int ps, int pn, int gl, int stride)
{
    const int64_t s = a.xadj[v];
    return dcut_sum_row(a, v, s, (int)(a.xadj[v + 1] - s), ps, pn, gl, stride);
}

__device__ __forceinline__ void move_meta(const KArgs &a, int v, int ps, int pn, int64_t &mw, uint64_t &dg)
{
    mw += a.vw ? a.vw[v] : 1;
    dg += mix64(((uint64_t)(uint32_t)v << 32) | (uint32_t)pn) - mix64(((uint64_t)(uint32_t)v << 32) | (uint32_t)ps);
}

template <int G>
__device__ void dcut_groups(const KArgs &a, int cls, int gid, int ngroups, int64_t &dc, int64_t &mw, uint64_t &dg,
                            int64_t &nm)
{
    const int gl = threadIdx.x & (G - 1);
    const int32_t *list = a.bins + a.binoff[cls];
    const int cnt = a.binoff[cls + 1] - a.binoff[cls];
    for (int i = gid; i < cnt; i += ngroups) {
        const int v = list[i];
        const int pn = a.dest[v];
        if (pn < 0) continue;
        const int ps = a.P[v];
        int d = dcut_sum(a, v, ps, pn, gl, G);
        d = gsum<G>(d);
        if (gl == 0) {
            dc += d;
            nm++;
            move_meta(a, v, ps, pn, mw, dg);
        }
    }
}

__global__ __launch_bounds__(BLOCK) void k_dcut(KArgs a)
{
    __shared__ int64_t s_red[BLOCK / 64];
    __shared__ uint64_t s_redu[BLOCK / 64];
    __shared__ int32_t s_red32[BLOCK / 64];
    __shared__ int32_t s_q[BLOCK];
    if (a.ctl->kind == KIND_DONE) return;
    // the previous iteration improved the best partition: copy P_iter before
    // this iteration's moves are applied
    if (a.ctl->copy_best)
        for (int v = blockIdx.x * BLOCK + threadIdx.x; v < a.n; v += gridDim.x * BLOCK) a.best[v] = a.P[v];
    int64_t dc = 0, mw = 0, nm = 0;
    uint64_t dg = 0;
    int b = blockIdx.x;
    if (b < a.gS) {
        int32_t *q = s_q + (threadIdx.x >> 6) * 64;
        wave_batched8(
            a.bins + a.binoff[CLS_S], a.binoff[CLS_S + 1] - a.binoff[CLS_S], q, b * (BLOCK / 64) + (threadIdx.x >> 6),
            a.gS * (BLOCK / 64),
            [&](Meta &m) -> bool {
                const int pn = a.dest[m.v];
                if (pn < 0) return false;
                m.aux = pn;
                m.ps = a.P[m.v];
                m.s = a.xadj[m.v];
                m.deg = (int)(a.xadj[m.v + 1] - m.s);
                return true;
            },
            [&](const Meta &t, int gl) {
                int d = dcut_sum_row(a, t.v, t.s, t.deg, t.ps, t.aux, gl, 8);
                d = gsum<8>(d);
                if (gl == 0) {
                    dc += d;
                    nm++;
                    move_meta(a, t.v, t.ps, t.aux, mw, dg);
                }
            });
    } else if ((b -= a.gS) < a.gM) {
        dcut_groups<64>(a, CLS_M, b * (BLOCK / 64) + (threadIdx.x >> 6), a.gM * (BLOCK / 64), dc, mw, dg, nm);
    } else if ((b -= a.gM) < a.gL) {
        const int32_t *list = a.bins + a.binoff[CLS_L];
        const int cnt = a.binoff[CLS_L + 1] - a.binoff[CLS_L];
        for (int i = b; i < cnt; i += a.gL) {
            const int v = list[i];
            const int pn = a.dest[v];
            if (pn < 0) continue;
            const int ps = a.P[v];
            int d = dcut_sum(a, v, ps, pn, threadIdx.x, BLOCK);
            d = block_sum<BLOCK>(d, s_red32);
            if (threadIdx.x == 0) { dc += d; nm++; move_meta(a, v, ps, pn, mw, dg); }
        }
    } else if ((b -= a.gL) < a.gZ) {
        const int32_t *list = a.bins + a.binoff[CLS_Z];
        const int cnt = a.binoff[CLS_Z + 1] - a.binoff[CLS_Z];
        for (int i = b * BLOCK + threadIdx.x; i < cnt; i += a.gZ * BLOCK) {
            const int v = list[i];
            const int pn = a.dest[v];
            if (pn < 0) continue;
            nm++;
            move_meta(a, v, a.P[v], pn, mw, dg);
        }
    }
    dc = block_sum<BLOCK>(dc, s_red);
    mw = block_sum<BLOCK>(mw, s_red);
    nm = block_sum<BLOCK>(nm, s_red);
    dg = block_sum<BLOCK>(dg, s_redu);
    if (threadIdx.x == 0) {
        shard_add(a, ST_DCUT, dc);
        shard_add(a, ST_MW, mw);
        shard_add(a, ST_M, nm);
        shard_add(a, ST_DIG, (int64_t)dg);
    }
}

// ------------------------------------------------------------ apply moves --

__global__ __launch_bounds__(BLOCK) void k_apply(KArgs a)
{
    extern __shared__ int32_t s_dw[];  // [k] block-partial weight change
    const int kind = a.ctl->kind;
    if (kind == KIND_DONE) return;
    for (int p = threadIdx.x; p < a.k; p += BLOCK) s_dw[p] = 0;
    __syncthreads();
    const int lp_id = a.ctl->lp_id;
    for (int v = blockIdx.x * BLOCK + threadIdx.x; v < a.n; v += gridDim.x * BLOCK) {
        const int pn = a.dest[v];
        if (pn < 0) continue;
        const int ps = a.P[v];
        const int vwv = a.vw ? a.vw[v] : 1;
        a.P[v] = pn;
        a.dest[v] = -1;
        if (kind == KIND_LP) a.lock[v] = lp_id;
        atomicSub(&s_dw[ps], vwv);
        atomicAdd(&s_dw[pn], vwv);
    }
    __syncthreads();
    for (int p = threadIdx.x; p < a.k; p += BLOCK)
        if (s_dw[p]) atomicAdd((unsigned long long *)&a.w[p], (unsigned long long)(int64_t)s_dw[p]);
}

// -------------------------------------------------------------- rebalance --

// Loss of an eligible vertex of an oversized part (Jetrw: own connectivity
// minus that of the best connected valid destination, ties -> smaller id, or
// a random valid destination when none is adjacent; Jetrs: own connectivity
// minus the floor mean over adjacent valid destinations), its slot, and the
// per-(part, slot) weight histogram.
__device__ __forceinline__ void rb_finish(const KArgs &a, int v, int ps, int vwv, int kind, uint64_t best, int cs,
                                          int sumB, int cntB, uint64_t hseed, int &ncand)
{
    int loss, d = -1;
    if (kind == KIND_RW) {
        if (best) {
            d = (int)(~(uint32_t)best);
            loss = cs - (int)(best >> 32);
        } else if (a.ctl->nB > 0) {
            const uint64_t h = mix64(hseed ^ (uint64_t)(uint32_t)v);
            d = a.Blist[__umul64hi(h, (uint64_t)a.ctl->nB)];
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
    ncand++;
    if (a.dbg_loss) { a.dbg_loss[v] = loss; a.dbg_slot[v] = s; a.dbg_pd[v] = d; }
}

__device__ __forceinline__ bool rb_eligible(const KArgs &a, int ps, int vwv)
{
    const int64_t k = a.k;
    return 2 * k * vwv <= 3 * (k * a.w[ps] - a.ctl->W);
}

template <int G, int R>
__device__ void rb_groups(const KArgs &a, int cls, int32_t *tab, int gid, int ngroups, int kind, uint64_t hseed,
                          int &ncand)
{
    const int gl = threadIdx.x & (G - 1);
    const int32_t *list = a.bins + a.binoff[cls];
    const int cnt = a.binoff[cls + 1] - a.binoff[cls];
    for (int i = gid; i < cnt; i += ngroups) {
        const int v = list[i];
        const int ps = a.P[v];
        const int vwv = a.vw ? a.vw[v] : 1;
        if (!a.isA[ps] || !rb_eligible(a, ps, vwv)) {
            if (gl == 0) { a.slot[v] = 255; if (a.dbg_loss) { a.dbg_loss[v] = INT64_MIN; a.dbg_slot[v] = -1; a.dbg_pd[v] = -1; } }
            continue;
        }
        int pu[R], cu[R];
        group_conn<G, R>(a, v, gl, tab, pu, cu);
        uint64_t best = 0;
        int cs = 0, sumB = 0, cntB = 0;
#pragma unroll
        for (int r = 0; r < R; r++) {
            if (cu[r] > 0) {
                if (pu[r] == ps) cs += cu[r];
                else if (a.isB[pu[r]]) {
                    uint64_t k2 = conn_key(cu[r], pu[r]);
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
        if (gl == 0) rb_finish(a, v, ps, vwv, kind, best, cs, sumB, cntB, hseed, ncand);
    }
}

__device__ void rb_blocks(const KArgs &a, int cls, int32_t *tab, int bid, int nblocks, int kind, uint64_t hseed,
                          int &ncand)
{
    __shared__ uint64_t s_red[BLOCK / 64];
    __shared__ int32_t s_red32[BLOCK / 64];
    const int32_t *list = a.bins + a.binoff[cls];
    const int cnt = a.binoff[cls + 1] - a.binoff[cls];
    for (int i = bid; i < cnt; i += nblocks) {
        const int v = list[i];
        const int ps = a.P[v];
        const int vwv = a.vw ? a.vw[v] : 1;
        if (!a.isA[ps] || !rb_eligible(a, ps, vwv)) {
            if (threadIdx.x == 0) { a.slot[v] = 255; if (a.dbg_loss) { a.dbg_loss[v] = INT64_MIN; a.dbg_slot[v] = -1; a.dbg_pd[v] = -1; } }
            continue;
        }
        block_fill(a, v, tab);
        uint64_t best = 0;
        int cs = 0, sumB = 0, cntB = 0;
        for (int p = threadIdx.x; p < a.k; p += BLOCK) {
            const int c = tab[p];
            if (c) {
                tab[p] = 0;
                if (p == ps) cs = c;
                else if (a.isB[p]) {
                    uint64_t k2 = conn_key(c, p);
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
        if (threadIdx.x == 0) rb_finish(a, v, ps, vwv, kind, best, cs, sumB, cntB, hseed, ncand);
    }
}

template <int ROLE, int GS = 8>
__global__ __launch_bounds__(BLOCK) void k_rb_loss(KArgs a, int nblk, int boff)
{
    extern __shared__ int32_t lds[];
    __shared__ int32_t s_red32[BLOCK / 64];
    const int kind = a.ctl->kind;
    if (kind != KIND_RW && kind != KIND_RS) return;
    const uint64_t hseed = mix64(a.ctl->seed ^ (((uint64_t)(uint32_t)a.ctl->level << 32) + (uint64_t)(uint32_t)a.ctl->t));
    const int stride = a.k + 1;
    int ncand = 0;
    if (ROLE == 1) {
        constexpr int RS_ = 32 / GS;
        const int ng = BLOCK / GS;
        for (int i = threadIdx.x; i < ng * stride; i += BLOCK) lds[i] = 0;
        __syncthreads();
        int32_t *tab = lds + (threadIdx.x / GS) * stride;
        int32_t *q = lds + ng * stride + (threadIdx.x >> 6) * 64;
        const int wid = blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6), nwaves = nblk * (BLOCK / 64);
        for (int c = 1; c < NCLS; c++) {
            if (a.tmap[c] != 1) continue;
            wave_batched<GS>(
                a.bins + a.binoff[c], a.binoff[c + 1] - a.binoff[c], q, wid, nwaves,
                [&](Meta &m) -> bool {
                    m.ps = a.P[m.v];
                    m.aux = a.vw ? a.vw[m.v] : 1;
                    if (!a.isA[m.ps] || !rb_eligible(a, m.ps, m.aux)) {
                        a.slot[m.v] = 255;
                        if (a.dbg_loss) { a.dbg_loss[m.v] = INT64_MIN; a.dbg_slot[m.v] = -1; a.dbg_pd[m.v] = -1; }
                        return false;
                    }
                    m.s = a.xadj[m.v];
                    m.deg = (int)(a.xadj[m.v + 1] - m.s);
                    return true;
                },
                [&](const Meta &t, int gl) {
                    int pu[RS_], cu[RS_];
                    group_conn_row<GS, RS_>(a, t.s, t.deg, gl, tab, pu, cu);
                    uint64_t best = 0;
                    int cs = 0, sumB = 0, cntB = 0;
#pragma unroll
                    for (int r = 0; r < RS_; r++) {
                        if (cu[r] > 0) {
                            if (pu[r] == t.ps) cs += cu[r];
                            else if (a.isB[pu[r]]) {
                                uint64_t k2 = conn_key(cu[r], pu[r]);
                                best = k2 > best ? k2 : best;
                                sumB += cu[r];
                                cntB++;
                            }
                        }
                    }
                    best = gmax_u64<GS>(best);
                    cs = gsum<GS>(cs);
                    sumB = gsum<GS>(sumB);
                    cntB = gsum<GS>(cntB);
                    if (gl == 0) rb_finish(a, t.v, t.ps, t.aux, kind, best, cs, sumB, cntB, hseed, ncand);
                });
        }
    } else if (ROLE == 2) {
        const int ng = BLOCK / 64;
        for (int i = threadIdx.x; i < ng * stride; i += BLOCK) lds[i] = 0;
        __syncthreads();
        int32_t *tab = lds + (threadIdx.x >> 6) * stride;
        for (int c = 1; c < NCLS; c++)
            if (a.tmap[c] == 2)
                rb_groups<64, 16>(a, c, tab, blockIdx.x * ng + (threadIdx.x >> 6), nblk * ng, kind, hseed, ncand);
    } else if (ROLE == 3) {
        for (int i = threadIdx.x; i < a.k; i += BLOCK) lds[i] = 0;
        __syncthreads();
        for (int c = 1; c < NCLS; c++)
            if (a.tmap[c] == 3) rb_blocks(a, c, lds, blockIdx.x, nblk, kind, hseed, ncand);
    } else {
        // isolated vertices: no connectivity, loss 0, random destination (Jetrw)
        const int32_t *list = a.bins + a.binoff[CLS_Z];
        const int cnt = a.binoff[CLS_Z + 1] - a.binoff[CLS_Z];
        for (int i = blockIdx.x * BLOCK + threadIdx.x; i < cnt; i += nblk * BLOCK) {
            const int v = list[i];
            const int ps = a.P[v];
            const int vwv = a.vw ? a.vw[v] : 1;
            if (!a.isA[ps] || !rb_eligible(a, ps, vwv)) {
                a.slot[v] = 255;
                if (a.dbg_loss) { a.dbg_loss[v] = INT64_MIN; a.dbg_slot[v] = -1; a.dbg_pd[v] = -1; }
                continue;
            }
            rb_finish(a, v, ps, vwv, kind, 0, 0, 0, 0, hseed, ncand);
        }
    }
    ncand = block_sum<BLOCK>(ncand, s_red32);
    if (threadIdx.x == 0) shard_add(a, ST_X, ncand);
}

// Per-(part, slot) weight histogram of the eligible vertices. Each block
// accumulates its grid-stride share in LDS when k * NSLOT int32 counters fit,
// then adds its nonzero counters to the global histogram.
__global__ __launch_bounds__(BLOCK) void k_rb_hist(KArgs a, int use_lds)
{
    extern __shared__ int32_t h[];
    const int kind = a.ctl->kind;
    if (kind != KIND_RW && kind != KIND_RS) return;
    const int nh = a.k * NSLOT;
    if (use_lds) {
        for (int i = threadIdx.x; i < nh; i += BLOCK) h[i] = 0;
        __syncthreads();
    }
    for (int v = blockIdx.x * BLOCK + threadIdx.x; v < a.n; v += gridDim.x * BLOCK) {
        const int sl = a.slot[v];
        if (sl == 255) continue;
        const int idx = a.P[v] * NSLOT + sl;
        const int vwv = a.vw ? a.vw[v] : 1;
        if (use_lds) atomicAdd(&h[idx], vwv);
        else atomicAdd((unsigned long long *)&a.hist[idx], (unsigned long long)(int64_t)vwv);
    }
    if (use_lds) {
        __syncthreads();
        for (int i = threadIdx.x; i < nh; i += BLOCK)
            if (h[i]) atomicAdd((unsigned long long *)&a.hist[i], (unsigned long long)(int64_t)h[i]);
    }
}

// Per oversized part: cut-off slot s* (slots below it are evicted whole) and
// the residual weight still needed inside s*; the compact list of parts whose
// cut-off lies inside the histogram; Jetrs capacities over B.
__global__ __launch_bounds__(BLOCK) void k_rb_cutoff(KArgs a)
{
    __shared__ int32_t s_scan[BLOCK / 64];
    __shared__ int64_t s_scan64[BLOCK / 64];
    Ctl *c = a.ctl;
    const int kind = c->kind;
    if (kind != KIND_RW && kind != KIND_RS) return;
    const int64_t o = c->o;
    int32_t carry = 0;
    for (int base = 0; base < a.k; base += BLOCK) {
        const int p = base + threadIdx.x;
        int split = 0;
        if (p < a.k) {
            int ss = -1;
            int64_t res = 0;
            if (a.isA[p]) {
                const int64_t need = a.w[p] - o;
                int64_t cum = 0;
                ss = NSLOT;
                for (int s = 0; s < NSLOT; s++) {
                    const int64_t h = a.hist[p * NSLOT + s];
                    if (cum + h >= need) { ss = s; res = need - cum; break; }
                    cum += h;
                }
            }
            a.sstar[p] = ss;
            a.resid[p] = res;
            split = ss >= 0 && ss < NSLOT;
        }
        int32_t tot;
        const int32_t pos = block_excl_scan<BLOCK>((int32_t)split, s_scan, tot);
        if (p < a.k) {
            a.splitidx[p] = split ? carry + pos : -1;
            if (split) a.splitpart[carry + pos] = p;
        }
        carry += tot;
    }
    if (threadIdx.x == 0) c->nsplit = carry;
    if (kind == KIND_RS) {
        const int nB = c->nB;
        const int64_t sigma = c->sigma;
        int64_t acc = 0;
        for (int base = 0; base < nB; base += BLOCK) {
            const int i = base + threadIdx.x;
            const int64_t cap = i < nB ? sigma - a.w[a.Blist[i]] : 0;
            int64_t tot;
            const int64_t pos = block_excl_scan<BLOCK>(cap, s_scan64, tot);
            if (i < nB) a.capstart[i] = acc + pos;
            acc += tot;
        }
        if (threadIdx.x == 0) { a.capstart[nB] = acc; c->total_cap = acc; }
    }
}

// Per tile of TILE vertices (one block) and split part j: weight of the
// tile's eligible vertices that sit in the part's cut-off slot, stored as
// tsum[j * ntile + tile].
__global__ __launch_bounds__(BLOCK) void k_rb_tilesum(KArgs a)
{
    extern __shared__ int32_t acc[];
    const int kind = a.ctl->kind;
    if (kind != KIND_RW && kind != KIND_RS) return;
    const int nsplit = a.ctl->nsplit;
    if (nsplit == 0) return;
    for (int tile = blockIdx.x; tile < a.ntile; tile += gridDim.x) {
        for (int j = threadIdx.x; j < nsplit; j += BLOCK) acc[j] = 0;
        __syncthreads();
        const int v0 = tile * TILE;
        for (int i = threadIdx.x; i < TILE; i += BLOCK) {
            const int v = v0 + i;
            if (v >= a.n) break;
            const int sl = a.slot[v];
            if (sl == 255) continue;
            const int p = a.P[v];
            if (sl == a.sstar[p]) atomicAdd(&acc[a.splitidx[p]], a.vw ? a.vw[v] : 1);
        }
        __syncthreads();
        for (int j = threadIdx.x; j < nsplit; j += BLOCK) a.tsum[(int64_t)j * a.ntile + tile] = acc[j];
        __syncthreads();
    }
}

// Per split part (one block): exclusive scan of its tile sums finds the one
// tile in which the running cut-off-slot weight reaches the residual (every
// cut-off-slot vertex of an earlier tile is evicted, none of a later one).
// Inside that tile the vertices are taken in id order while the weight
// before them is below the residual; the last evicted id is the threshold.
__global__ __launch_bounds__(BLOCK) void k_rb_split(KArgs a)
{
    __shared__ int64_t s_scan[BLOCK / 64];
    __shared__ uint64_t s_red[BLOCK / 64];
    __shared__ int s_tile;
    __shared__ int64_t s_base;
    constexpr int PER = TILE / BLOCK;
    const int kind = a.ctl->kind;
    if (kind != KIND_RW && kind != KIND_RS) return;
    const int nsplit = a.ctl->nsplit;
    for (int j = blockIdx.x; j < nsplit; j += gridDim.x) {
        const int p = a.splitpart[j];
        const int32_t *row = a.tsum + (int64_t)j * a.ntile;
        const int64_t resid = a.resid[p];
        int64_t carry = 0;
        for (int b0 = 0; b0 < a.ntile; b0 += BLOCK) {
            const int i = b0 + threadIdx.x;
            const int64_t x = i < a.ntile ? row[i] : 0;
            int64_t tot;
            const int64_t before = carry + block_excl_scan<BLOCK>(x, s_scan, tot);
            if (x > 0 && before < resid && resid <= before + x) { s_tile = i; s_base = before; }
            carry += tot;
        }
        __syncthreads();
        const int ss = a.sstar[p];
        const int v0 = s_tile * TILE + threadIdx.x * PER;
        int wv[PER];
        int64_t mine = 0;
#pragma unroll
        for (int q = 0; q < PER; q++) {
            const int v = v0 + q;
            wv[q] = 0;
            if (v < a.n && a.slot[v] == ss && a.P[v] == p) wv[q] = a.vw ? a.vw[v] : 1;
            mine += wv[q];
        }
        int64_t tot;
        int64_t before = s_base + block_excl_scan<BLOCK>(mine, s_scan, tot);
        uint64_t last = 0;  // (last evicted id + 1), 0 = none
#pragma unroll
        for (int q = 0; q < PER; q++) {
            if (wv[q] > 0 && before < resid) last = (uint64_t)(v0 + q) + 1;
            before += wv[q];
        }
        last = block_max_u64<BLOCK>(last, s_red);
        if (threadIdx.x == 0) a.vthr[p] = (int32_t)last - 1;
        __syncthreads();
    }
}

// Eviction decision for every eligible vertex (one block per tile): evicted
// when its slot is below the part's cut-off, or equal with an id no larger
// than the part's threshold. Jetrw moves it to its chosen destination; Jetrs
// marks it and sums the tile's evicted weight.
__global__ __launch_bounds__(BLOCK) void k_rb_mark(KArgs a)
{
    __shared__ int64_t s_red[BLOCK / 64];
    const int kind = a.ctl->kind;
    if (kind != KIND_RW && kind != KIND_RS) return;
    for (int tile = blockIdx.x; tile < a.ntile; tile += gridDim.x) {
        int64_t esum = 0;
        const int v0 = tile * TILE;
        for (int i = threadIdx.x; i < TILE; i += BLOCK) {
            const int v = v0 + i;
            if (v >= a.n) break;
            const int sl = a.slot[v];
            bool ev = false;
            if (sl != 255) {
                const int p = a.P[v];
                const int ss = a.sstar[p];
                ev = sl < ss || (sl == ss && v <= a.vthr[p]);
            }
            if (kind == KIND_RW) {
                if (ev) a.dest[v] = a.rbd[v];
            } else {
                a.rsev[v] = ev;
                if (ev) esum += a.vw ? a.vw[v] : 1;
            }
        }
        if (kind == KIND_RS) {
            esum = block_sum<BLOCK>(esum, s_red);
            if (threadIdx.x == 0) a.esum[tile] = esum;
        }
    }
}

// Jetrs: exclusive scan of the evicted weight over tiles.
__global__ __launch_bounds__(BLOCK) void k_rs_scan(KArgs a)
{
    __shared__ int64_t s_scan[BLOCK / 64];
    if (a.ctl->kind != KIND_RS) return;
    int64_t carry = 0;
    for (int base = 0; base < a.ntile; base += BLOCK) {
        const int i = base + threadIdx.x;
        const int64_t x = i < a.ntile ? a.esum[i] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan<BLOCK>(x, s_scan, tot);
        if (i < a.ntile) a.esum[i] = carry + ex;
        carry += tot;
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
    constexpr int PER = TILE / BLOCK;
    if (a.ctl->kind != KIND_RS) return;
    const int nB = a.ctl->nB;
    const int64_t total = a.ctl->total_cap;
    for (int tile = blockIdx.x; tile < a.ntile; tile += gridDim.x) {
        const int v0 = tile * TILE + threadIdx.x * PER;
        int wv[PER];
        int64_t mine = 0;
#pragma unroll
        for (int q = 0; q < PER; q++) {
            const int v = v0 + q;
            wv[q] = (v < a.n && a.rsev[v]) ? (a.vw ? a.vw[v] : 1) : 0;
            mine += wv[q];
        }
        int64_t tot;
        int64_t pos = a.esum[tile] + block_excl_scan<BLOCK>(mine, s_scan, tot);
#pragma unroll
        for (int q = 0; q < PER; q++) {
            if (wv[q] > 0 && pos < total) {
                int lo = 0, hi = nB;  // largest i with capstart[i] <= pos (capstart[0] = 0 <= pos)
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (a.capstart[mid] <= pos) lo = mid; else hi = mid;
                }
                a.dest[v0 + q] = a.Blist[lo];
            }
            pos += wv[q];
        }
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
    Buffer &b = ctx->bufs[slot];
    if (b.bytes >= bytes) return b.ptr;
    if (b.ptr) { (void)hipFree(b.ptr); b.ptr = nullptr; b.bytes = 0; }
    size_t want = bytes + bytes / 8;  // headroom for the next, slightly larger level
    if (hipMalloc(&b.ptr, want) != hipSuccess) {
        (void)hipGetLastError();
        b.ptr = nullptr;
        return nullptr;
    }
    b.bytes = want;
    return b.ptr;
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

struct Plan {
    KArgs tab;    // LDS-table kernels (gain, loss)
    KArgs plain;  // afterburner, cut delta
    int grid_tab, grid_plain, grid_rbtab;
    size_t lds_tab;
    int grid_flat;
    int grid_tile;
    int grid_hist;
    bool hist_lds;
};

static int div_up(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

static void plan_roles(const jet_context *ctx, KArgs &a, const int32_t *cnt, Plan &pl)
{
    const int maxb = ctx->num_cu * 8;
    // LDS-table kernels: the 8-lane role keeps 32 tables of k ints, the wave
    // role 4, the block role 1; larger k moves classes to roles with fewer
    // tables so a block stays within 64 KiB of LDS.
    KArgs t = a;
    t.tmap[0] = 0;
    const int k = a.k;
    if (k <= 495) { t.tmap[1] = 1; t.tmap[2] = 2; t.tmap[3] = 3; }
    else if (k <= 4095) { t.tmap[1] = 2; t.tmap[2] = 2; t.tmap[3] = 3; }
    else { t.tmap[1] = 3; t.tmap[2] = 3; t.tmap[3] = 3; }
    int64_t role_cnt[4] = {0, 0, 0, 0};
    for (int c = 1; c < NCLS; c++) role_cnt[t.tmap[c]] += cnt[c];
    t.gS = std::min(div_up(role_cnt[1], BLOCK / 8), maxb);
    t.gM = std::min(div_up(role_cnt[2], BLOCK / 64), maxb);
    t.gL = std::min((int)role_cnt[3], maxb);
    t.gZ = std::min(div_up(cnt[0], BLOCK), maxb);
    size_t lds = 0;
    if (t.gS) lds = std::max(lds, (size_t)(BLOCK / 8) * k * 4);
    if (t.gM) lds = std::max(lds, (size_t)(BLOCK / 64) * k * 4);
    if (t.gL) lds = std::max(lds, (size_t)k * 4);
    pl.lds_tab = lds;
    pl.grid_tab = t.gS + t.gM + t.gL;       // gain: no isolated role
    pl.grid_rbtab = t.gS + t.gM + t.gL + t.gZ;
    // plain row kernels: roles follow the classes directly
    KArgs p = a;
    p.tmap[0] = 0; p.tmap[1] = 1; p.tmap[2] = 2; p.tmap[3] = 3;
    p.gS = std::min(div_up(cnt[1], BLOCK / 8), maxb);
    p.gM = std::min(div_up(cnt[2], BLOCK / 64), maxb);
    p.gL = std::min(cnt[3], maxb);
    p.gZ = std::min(div_up(cnt[0], BLOCK), maxb);
    pl.grid_plain = p.gS + p.gM + p.gL + p.gZ;
    for (KArgs *x : {&t, &p}) {
        x->grid_tab = pl.grid_tab;
        x->grid_rbtab = pl.grid_rbtab;
        x->grid_plain = pl.grid_plain;
    }
    pl.tab = t;
    pl.plain = p;
    pl.hist_lds = (size_t)a.k * NSLOT * 4 <= 65536;
    pl.grid_hist = std::max(1, std::min(a.ntile, ctx->num_cu * 2));
    pl.grid_flat = std::max(1, std::min(div_up(a.n, BLOCK), ctx->num_cu * 2));
    pl.grid_tile = std::max(1, std::min(a.ntile, ctx->num_cu * 8));
}

// Up to this k the 8-lane role runs with 4 lanes per vertex (64 tables of
// k + 1 ints per block fit in 32 KiB): twice the vertices in flight per wave.
constexpr int K_G4 = 120;

static void launch_gain(const Plan &pl, hipStream_t s)
{
    const KArgs &t = pl.tab;
    const size_t st = (size_t)(t.k + 1) * 4;
    if (t.gS) {
        if (t.k <= K_G4) k_gain<1, 4><<<t.gS, BLOCK, (BLOCK / 4) * st + BLOCK * 4, s>>>(t, t.gS, 0);
        else k_gain<1, 8><<<t.gS, BLOCK, (BLOCK / 8) * st + BLOCK * 4, s>>>(t, t.gS, 0);
    }
    if (t.gM) k_gain<2><<<t.gM, BLOCK, (BLOCK / 64) * st, s>>>(t, t.gM, t.gS);
    if (t.gL) k_gain<3><<<t.gL, BLOCK, (size_t)t.k * 4, s>>>(t, t.gL, t.gS + t.gM);
}

static void launch_rb_loss(const Plan &pl, hipStream_t s)
{
    const KArgs &t = pl.tab;
    const size_t st = (size_t)(t.k + 1) * 4;
    if (t.gS) {
        if (t.k <= K_G4) k_rb_loss<1, 4><<<t.gS, BLOCK, (BLOCK / 4) * st + BLOCK * 4, s>>>(t, t.gS, 0);
        else k_rb_loss<1, 8><<<t.gS, BLOCK, (BLOCK / 8) * st + BLOCK * 4, s>>>(t, t.gS, 0);
    }
    if (t.gM) k_rb_loss<2><<<t.gM, BLOCK, (BLOCK / 64) * st, s>>>(t, t.gM, t.gS);
    if (t.gL) k_rb_loss<3><<<t.gL, BLOCK, (size_t)t.k * 4, s>>>(t, t.gL, t.gS + t.gM);
    if (t.gZ) k_rb_loss<4><<<t.gZ, BLOCK, 0, s>>>(t, t.gZ, t.gS + t.gM + t.gL);
}

// Histogram, cut-off slots, ordered selection and (Jetrs) the cookie-cutter.
static void launch_rb_select(const Plan &pl, hipStream_t s)
{
    const KArgs &p = pl.plain;
    k_rb_hist<<<pl.grid_hist, BLOCK, pl.hist_lds ? (size_t)p.k * NSLOT * 4 : 0, s>>>(p, pl.hist_lds);
    k_rb_cutoff<<<1, BLOCK, 0, s>>>(p);
    k_rb_tilesum<<<pl.grid_tile, BLOCK, (size_t)p.k * 4, s>>>(p);
    k_rb_split<<<std::min(p.k, 1024), BLOCK, 0, s>>>(p);
    k_rb_mark<<<pl.grid_tile, BLOCK, 0, s>>>(p);
    k_rs_scan<<<1, BLOCK, 0, s>>>(p);
    k_rs_assign<<<pl.grid_tile, BLOCK, 0, s>>>(p);
}

static void launch_iteration(const Plan &pl, hipStream_t s, bool lp_kernels, bool rb_kernels,
                             hipEvent_t ev_a = nullptr, hipEvent_t ev_b = nullptr)
{
    const KArgs &p = pl.plain;
    if (lp_kernels) {
        if (ev_a) (void)hipEventRecord(ev_a, s);
        launch_gain(pl, s);
        if (ev_b) (void)hipEventRecord(ev_b, s);
        if (pl.grid_plain) k_afterburner<<<pl.grid_plain, BLOCK, 0, s>>>(p);
    }
    if (rb_kernels) {
        launch_rb_loss(pl, s);
        launch_rb_select(pl, s);
    }
    if (pl.grid_plain) k_dcut<<<pl.grid_plain, BLOCK, 0, s>>>(p);
    k_apply<<<pl.grid_flat, BLOCK, (size_t)p.k * 4, s>>>(p);
    k_ctl_end<<<1, CTL_NT, 0, s>>>(p);
}

static void set_lds_limits()
{
    static bool done = false;
    if (done) return;
    done = true;
    (void)hipFuncSetAttribute((const void *)k_gain<1, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_gain<1, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_gain<2>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_gain<3>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_rb_loss<1, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_rb_loss<1, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_rb_loss<2>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_rb_loss<3>, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_apply, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_init_vertices, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_rb_tilesum, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    (void)hipFuncSetAttribute((const void *)k_rb_hist, hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
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
    JET_TRY(hipStreamSynchronize(s));
    if (xadj[0] != 0 || xadj[n] != nnz) return JET_EGRAPH;
    std::vector<uint64_t> key(nnz), rkey(nnz);
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

// Shared set-up of a refinement call: validates, fills the workspace and the
// controller, and returns the launch plan.
static int setup(jet_context *ctx, const jet_csr *g, const jet_params *prm, int32_t *part, Plan &pl,
                 Ctl &hc, hipStream_t s, jet_trace_rec *trace_dev, int32_t trace_cap, const DebugOut *dbg)
{
    const int n = g->n, k = prm->k;
    set_lds_limits();
    if (prm->flags & JET_F_VALIDATE) {
        int st = validate_full_csr(ctx, g, s);
        if (st) return st;
    }
    KArgs a;
    memset(&a, 0, sizeof(a));
    a.n = n; a.k = k;
    a.xadj = g->xadj; a.adj = g->adjncy; a.vw = g->vwgt; a.ew = g->adjwgt;
    const size_t nn = (size_t)std::max(n, 1);
    a.P = (int32_t *)ws_get(ctx, WS_P, nn * 4);
    a.rec = (int2 *)ws_get(ctx, WS_REC, nn * 8);
    a.dest = (int32_t *)ws_get(ctx, WS_DEST, nn * 4);
    a.lock = (int32_t *)ws_get(ctx, WS_LOCK, nn * 4);
    a.slot = (uint8_t *)ws_get(ctx, WS_SLOT, nn);
    a.rbd = (int32_t *)ws_get(ctx, WS_RBD, nn * 4);
    a.rsev = (uint8_t *)ws_get(ctx, WS_RSEV, nn);
    int32_t *bins = (int32_t *)ws_get(ctx, WS_BIN, nn * 4);
    a.bins = bins;
    a.bstat = (int64_t *)ws_get(ctx, WS_BSTAT, sizeof(int64_t) * NSTAT * NSHARD);
    int32_t *fill = (int32_t *)ws_get(ctx, WS_FILL, sizeof(int32_t) * NCLS);
    a.ctl = (Ctl *)ws_get(ctx, WS_CTL, sizeof(Ctl) + 64);
    int64_t *p64 = (int64_t *)ws_get(ctx, WS_PART64, sizeof(int64_t) * (5 * (size_t)k + 8));
    int32_t *p32 = (int32_t *)ws_get(ctx, WS_PART32, sizeof(int32_t) * (6 * (size_t)k + 8));
    uint8_t *p8 = (uint8_t *)ws_get(ctx, WS_PART8, 2 * (size_t)k + 16);
    a.hist = (int64_t *)ws_get(ctx, WS_HIST, sizeof(int64_t) * (size_t)k * NSLOT);
    a.ntile = std::max(1, div_up(n, TILE));
    a.tsum = (int32_t *)ws_get(ctx, WS_TSUM, sizeof(int32_t) * (size_t)a.ntile * k);
    a.esum = (int64_t *)ws_get(ctx, WS_ESUM, sizeof(int64_t) * (size_t)a.ntile);
    a.kinds = (int8_t *)ws_get(ctx, WS_KINDS, KIND_LOG);
    if (!a.P || !a.rec || !a.dest || !a.lock || !a.slot || !a.rbd || !a.rsev || !bins || !a.bstat || !fill ||
        !a.ctl || !p64 || !p32 || !p8 || !a.hist || !a.tsum || !a.esum || !a.kinds)
        return JET_ENOMEM;
    a.w = p64; a.wbest = p64 + k; a.resid = p64 + 2 * k; a.xbase = p64 + 3 * k; a.capstart = p64 + 4 * k;
    a.Blist = p32; a.sstar = p32 + k; a.splitidx = p32 + 2 * k; a.splitpart = p32 + 3 * k; a.xtile = p32 + 4 * k;
    a.vthr = p32 + 5 * k;
    a.isA = p8; a.isB = p8 + k;
    a.best = part;
    a.trace = trace_dev;
    if (dbg) {
        a.dbg_F = dbg->F; a.dbg_cs = dbg->cs; a.dbg_F2 = dbg->F2; a.dbg_loss = dbg->loss;
        a.dbg_pd = dbg->pd; a.dbg_slot = dbg->slot;
    }
    // controller configuration; state starts at zero
    memset(&hc, 0, sizeof(hc));
    hc.n = n; hc.k = k;
    hc.stall_limit = prm->stall_limit > 0 ? prm->stall_limit : 12;
    hc.bmax = prm->weak_rebalance_iters == 0 ? 2 : (prm->weak_rebalance_iters < 0 ? 0 : prm->weak_rebalance_iters);
    hc.max_iters = prm->max_iters;
    if (prm->c_den > 0) { hc.c_num = prm->c_num; hc.c_den = prm->c_den; }
    else { hc.c_num = prm->level == 0 ? 1 : 3; hc.c_den = 4; }
    hc.phi_num = prm->phi_num > 0 ? prm->phi_num : 999;
    hc.phi_den = prm->phi_den > 0 ? prm->phi_den : 1000;
    hc.level = prm->level;
    hc.trace_cap = trace_dev ? trace_cap : 0;
    hc.seed = prm->seed;
    Ctl *pin = (Ctl *)ctx->pinned;
    *pin = hc;
    JET_TRY(hipMemcpyAsync(a.ctl, pin, sizeof(Ctl), hipMemcpyHostToDevice, s));
    JET_TRY(hipMemsetAsync(a.w, 0, sizeof(int64_t) * k, s));
    const int grid_v = std::max(1, std::min(div_up(n, BLOCK), ctx->num_cu * 4));
    if (n > 0) k_init_vertices<<<grid_v, BLOCK, (size_t)k * 4, s>>>(a, part);
    if (g->nnz > 0) {
        const int grid_e = std::max(1, std::min(div_up(div_up(g->nnz, 16), BLOCK), ctx->num_cu * 8));
        k_init_edges<<<grid_e, BLOCK, 0, s>>>(a, g->nnz);
    }
    JET_TRY(hipGetLastError());
    JET_TRY(hipMemcpyAsync(pin, a.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
    int64_t *xends = (int64_t *)((char *)ctx->pinned + 2048);
    JET_TRY(hipMemcpyAsync(xends, g->xadj, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    JET_TRY(hipMemcpyAsync(xends + 1, g->xadj + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    JET_TRY(hipStreamSynchronize(s));
    hc = *pin;
    if (xends[0] != 0 || xends[1] != g->nnz) return JET_EGRAPH;
    if (hc.bad_graph) return JET_EGRAPH;
    if (hc.bad_part) return JET_EPART;
    if (hc.wsum >= ((int64_t)1 << 31) || hc.ewsum >= ((int64_t)1 << 31)) return JET_EOVERFLOW;
    a.binoff[0] = 0;
    for (int c = 0; c < NCLS; c++) a.binoff[c + 1] = a.binoff[c] + hc.bincnt[c];
    JET_TRY(hipMemsetAsync(fill, 0, sizeof(int32_t) * NCLS, s));
    if (n > 0) k_fill_bins<<<grid_v, BLOCK, 0, s>>>(a, bins, fill);
    const int64_t W = hc.wsum;
    const int64_t o = balance_limit(W, k, prm->lambda_ppm);
    const int64_t sigma = deadzone_sigma(W, k, o, prm->deadzone_div > 0 ? prm->deadzone_div : 10);
    k_ctl_setup<<<1, BLOCK, 0, s>>>(a, W, o, sigma);
    JET_TRY(hipGetLastError());
    hc.W = W; hc.o = o; hc.sigma = sigma;
    plan_roles(ctx, a, hc.bincnt, pl);
    return JET_OK;
}

int refine_level(jet_context *ctx, const jet_csr *g, const jet_params *prm, int32_t *part,
                 int64_t *part_weights_out, jet_stats *stats, jet_trace_rec *trace_host, int32_t trace_cap,
                 int32_t *trace_count, int32_t *trace_total, hipStream_t s)
{
    int st = check_params(g, prm);
    if (st) return st;
    const int n = g->n, k = prm->k;
    if (trace_count) *trace_count = 0;
    if (trace_total) *trace_total = 0;
    JET_TRY(hipEventRecord(ctx->ev[0], s));
    if (k == 1 || n == 0) {
        // a single part: every vertex in part 0, nothing to refine
        if (n > 0) JET_TRY(hipMemsetAsync(part, 0, sizeof(int32_t) * n, s));
        int64_t W = n;
        if (n > 0 && g->vwgt) {
            std::vector<int32_t> vw(n);
            JET_TRY(hipMemcpyAsync(vw.data(), g->vwgt, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
            JET_TRY(hipStreamSynchronize(s));
            W = 0;
            for (int32_t x : vw) W += x;
        }
        if (part_weights_out) {
            std::vector<int64_t> pw(k, 0);
            pw[0] = W;
            JET_TRY(hipMemcpyAsync(part_weights_out, pw.data(), sizeof(int64_t) * k, hipMemcpyHostToDevice, s));
        }
        JET_TRY(hipStreamSynchronize(s));
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
    jet_trace_rec *trace_dev = nullptr;
    if (trace_host && trace_cap > 0) {
        trace_dev = (jet_trace_rec *)ws_get(ctx, WS_TRACE, sizeof(jet_trace_rec) * (size_t)trace_cap);
        if (!trace_dev) return JET_ENOMEM;
    }
    Plan pl;
    Ctl hc;
    st = setup(ctx, g, prm, part, pl, hc, s, trace_dev, trace_cap, nullptr);
    if (st) return st;
    JET_TRY(hipEventRecord(ctx->ev[1], s));
    Ctl *pin = (Ctl *)ctx->pinned;
    const bool prof = prm->flags & JET_F_PROFILE;
    int chunk = 4, launched = 0;
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
            launch_iteration(pl, s, true, true, ea, eb);
            launched++;
        }
        JET_TRY(hipGetLastError());
        JET_TRY(hipMemcpyAsync(pin, pl.plain.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s));
        JET_TRY(hipStreamSynchronize(s));
        if (pin->done) break;
        chunk = std::min(chunk * 2, 32);
    }
    hc = *pin;
    k_copy_best<<<pl.grid_flat, BLOCK, 0, s>>>(pl.plain);
    JET_TRY(hipEventRecord(ctx->ev[2], s));
    if (prm->flags & JET_F_RETURN_ITER)
        JET_TRY(hipMemcpyAsync(part, pl.plain.P, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    if (part_weights_out)
        JET_TRY(hipMemcpyAsync(part_weights_out, (prm->flags & JET_F_RETURN_ITER) ? pl.plain.w : pl.plain.wbest,
                               sizeof(int64_t) * k, hipMemcpyDeviceToDevice, s));
    const int ntr = std::min(hc.t, hc.trace_cap);
    if (trace_dev && ntr > 0)
        JET_TRY(hipMemcpyAsync(trace_host, trace_dev, sizeof(jet_trace_rec) * ntr, hipMemcpyDeviceToHost, s));
    JET_TRY(hipEventRecord(ctx->ev[3], s));
    JET_TRY(hipStreamSynchronize(s));
    if (trace_count) *trace_count = ntr;
    if (trace_total) *trace_total = hc.t;
    float ms_gain = 0.f;
    int gain_passes = 0;
    if (prof) {
        const int nk = std::min(hc.t, KIND_LOG);
        std::vector<int8_t> kinds(std::max(nk, 1));
        if (nk > 0) {
            JET_TRY(hipMemcpyAsync(kinds.data(), pl.plain.kinds, nk, hipMemcpyDeviceToHost, s));
            JET_TRY(hipStreamSynchronize(s));
        }
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
        memset(stats, 0, sizeof(*stats));
        const bool it = prm->flags & JET_F_RETURN_ITER;
        stats->cut = it ? hc.cut : hc.cut_best;
        stats->max_part_weight = it ? hc.maxw : hc.maxw_best;
        stats->o = hc.o;
        stats->sigma = hc.sigma;
        stats->total_weight = hc.W;
        stats->balanced = stats->max_part_weight <= hc.o;
        stats->iters = hc.t;
        stats->lp_iters = hc.n_lp;
        stats->rw_iters = hc.n_rw;
        stats->rs_iters = hc.n_rs;
        stats->levels = 1;
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

}  // namespace jet

using namespace jet;

// --------------------------------------------------------------- C ABI ------

extern "C" int jet_context_create(jet_context **out, int device)
{
    if (!out) return JET_EINVAL;
    *out = nullptr;
    jet_context *ctx = new (std::nothrow) jet_context();
    if (!ctx) return JET_ENOMEM;
    ctx->device = device;
    ctx->bufs.resize(WS_COUNT);
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) { int st = hip_status(ctx, e); delete ctx; return st; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        ctx->num_cu = prop.multiProcessorCount;
    ctx->pinned_bytes = 4096;
    e = hipHostMalloc(&ctx->pinned, ctx->pinned_bytes, hipHostMallocDefault);
    if (e != hipSuccess) { int st = hip_status(ctx, e); delete ctx; return st; }
    for (auto &ev : ctx->ev) {
        e = hipEventCreate(&ev);
        if (e != hipSuccess) { int st = hip_status(ctx, e); jet_context_destroy(ctx); return st; }
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
    case JET_EOVERFLOW: return "total vertex or edge weight too large (>= 2^31)";
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
    int32_t cnt = 0, tot = 0;
    int st = refine_level(ctx, g, params, part, part_weights_out, stats, trace ? trace->recs : nullptr,
                          trace ? trace->cap : 0, &cnt, &tot, (hipStream_t)stream);
    if (trace) { trace->count = cnt; trace->total = tot; }
    return st;
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
    // private copy of the partition: the step leaves `part` untouched
    int32_t *p0 = (int32_t *)ws_get(ctx, WS_H0, sizeof(int32_t) * n);
    if (!p0) return JET_ENOMEM;
    JET_TRY(hipMemcpyAsync(p0, part, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    DebugOut dbg;
    dbg.F = F; dbg.cs = conn_s; dbg.F2 = F2; dbg.pd = pd;
    Plan pl;
    Ctl hc;
    st = setup(ctx, g, params, p0, pl, hc, s, nullptr, 0, &dbg);
    if (st) return st;
    k_step_defaults<<<pl.grid_flat, BLOCK, 0, s>>>(pl.plain, part);
    k_force_step<<<pl.grid_flat, BLOCK, 0, s>>>(pl.plain, KIND_LP, 0, locked);
    launch_gain(pl, s);
    if (pl.grid_plain) k_afterburner<<<pl.grid_plain, BLOCK, 0, s>>>(pl.plain);
    k_lp_outputs<<<pl.grid_flat, BLOCK, 0, s>>>(pl.plain, inX, move);
    JET_TRY(hipGetLastError());
    JET_TRY(hipStreamSynchronize(s));
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
    int32_t *p0 = (int32_t *)ws_get(ctx, WS_H0, sizeof(int32_t) * n);
    int32_t *pdv = (int32_t *)ws_get(ctx, WS_DBG_LOCK, sizeof(int32_t) * n);
    if (!p0 || !pdv) return JET_ENOMEM;
    JET_TRY(hipMemcpyAsync(p0, part, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    DebugOut dbg;
    dbg.loss = loss; dbg.slot = slot; dbg.pd = pdv;
    Plan pl;
    Ctl hc;
    st = setup(ctx, g, params, p0, pl, hc, s, nullptr, 0, &dbg);
    if (st) return st;
    const KArgs &p = pl.plain;
    k_step_defaults<<<pl.grid_flat, BLOCK, 0, s>>>(p, part);
    k_force_step<<<1, BLOCK, 0, s>>>(p, kind, t, nullptr);
    launch_rb_loss(pl, s);
    launch_rb_select(pl, s);
    JET_TRY(hipGetLastError());
    JET_TRY(hipMemcpyAsync(dest, p.dest, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    JET_TRY(hipStreamSynchronize(s));
    return JET_OK;
}
