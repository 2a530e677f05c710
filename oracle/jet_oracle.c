/*
 * Jet refinement oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded C implementation of what the Jet
 * refinement pass computes (Gilbert, Madduri, Boman, Rajamanickam,
 * "Jet: Multilevel Graph Partitioning on Graphics Processing Units"):
 *   - the refinement loop of Algorithm 3 (Section 4),
 *   - Jetlp with its first filter and the afterburner (Algorithm 4,
 *     Section 4.1, the ord relation and eq. gainconn_filter),
 *   - weak rebalancing Jetrw (Algorithm 5, Section 4.2.2) and strong
 *     rebalancing Jetrs (Section 4.2.2, the "cookie-cutter" overlay),
 *   - the loss slot function of Section 4.2.1,
 *   - and, as the multilevel scaffold, heavy-edge matching, contraction
 *     (Algorithm 2), projection and a seeded random coarsest partition
 *     (Algorithm 1).
 * Everything is recomputed from scratch: connectivity is a dense k-array per
 * vertex, part weights and the cut are recomputed by brute force after every
 * iteration. Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark call this code; the product path never does.
 *
 * Integer arithmetic throughout: int32 weights, int64 gains, losses, cuts and
 * part weights. Readings of points the paper leaves open are marked
 * "reading:" below.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n;
    const int64_t *xadj;   /* [n+1] */
    const int32_t *adjncy; /* [xadj[n]] */
    const int32_t *vwgt;   /* [n] */
    const int32_t *adjwgt; /* [xadj[n]] */
} og_graph;

typedef struct {
    int32_t k;
    int32_t lambda_ppm;      /* imbalance lambda in parts per million */
    int32_t c_num, c_den;    /* first-filter ratio c; c_den == 0 -> 1/4 at level 0, 3/4 above */
    int32_t phi_num, phi_den;/* tolerance phi, 999/1000 */
    int32_t stall_limit;     /* 12 */
    int32_t bmax;            /* weak rebalance iterations before strong: 2 */
    int32_t deadzone_div;    /* sigma rule divisor: 10 */
    int32_t level;
    int32_t max_iters;       /* 0 = no cap */
    int32_t flags;           /* OG_F_* (Jetlp ablations) */
    uint64_t seed;
} og_params;

/* Jetlp ablations of Section 7.1 (Component Effectiveness, Table lp_versions).
 * Reading: "ignores the lock bit" = R stays empty; "omits the afterburner"
 * = every vertex of X moves (F2 is left 0). The weak afterburner (moves with
 * F >= 0 only) is the first filter with c = 0. Bit values follow the public
 * flags of the library's interface. */
#define OG_F_NO_LOCKS 0x8
#define OG_F_NO_AFTERBURNER 0x10
/* coarsening with two-hop matching (Section 3.1) after heavy-edge matching */
#define OG_F_TWO_HOP 0x20
/* graph-growing start of the coarsest graph (og_bfs_part) instead of the
 * seeded random one */
#define OG_F_BFS_START 0x40

typedef struct {
    int32_t level, t, kind, nX, nM, stall, wcount, balanced;
    int64_t moved_w, cut, maxw, best_cut;
    uint64_t digest;
} og_trace;

enum { OG_LP = 1, OG_RW = 2, OG_RS = 3 };

/* ---- SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) ---------------------- */
static uint64_t og_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static uint64_t og_stream(uint64_t seed, uint64_t i)
{
    return og_mix64(seed + (i + 1) * 0x9E3779B97F4A7C15ULL);
}
static uint64_t og_below(uint64_t x, uint64_t r)
{
    return (uint64_t)(((unsigned __int128)x * r) >> 64);
}

/* ---- definitions of Section 2.1 ---------------------------------------- */
static int64_t og_total_weight(const og_graph *g)
{
    int64_t W = 0;
    for (int32_t v = 0; v < g->n; v++) W += g->vwgt[v];
    return W;
}

static void og_part_weights(const og_graph *g, const int32_t *P, int32_t k, int64_t *w)
{
    for (int32_t p = 0; p < k; p++) w[p] = 0;
    for (int32_t v = 0; v < g->n; v++) w[P[v]] += g->vwgt[v];
}

/* cut = sum over undirected edges {u,v} with P(u) != P(v) of w_uv; every
 * edge is stored twice, so count it from its smaller endpoint. */
static int64_t og_cut(const og_graph *g, const int32_t *P)
{
    int64_t c = 0;
    for (int32_t v = 0; v < g->n; v++)
        for (int64_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
            int32_t u = g->adjncy[e];
            if (u > v && P[u] != P[v]) c += g->adjwgt[e];
        }
    return c;
}

static int64_t og_max(const int64_t *w, int32_t k)
{
    int64_t m = w[0];
    for (int32_t p = 1; p < k; p++) if (w[p] > m) m = w[p];
    return m;
}

/* balance limit o = floor((1 + lambda) W / k), lambda as integer ppm. */
static int64_t og_limit(int64_t W, int32_t k, int32_t lambda_ppm)
{
    __int128 num = (__int128)W * (1000000 + (__int128)lambda_ppm);
    return (int64_t)(num / ((__int128)k * 1000000));
}

/* Deadzone bound sigma (maxDestSize in Algorithm 5). The paper only asks for
 * a deadzone between sigma and o. reading: slack = o - ceil(W/k);
 * slack <= 0 -> o; slack < div -> o - 1; else o - floor(slack / div). */
static int64_t og_sigma(int64_t W, int32_t k, int64_t o, int32_t div)
{
    int64_t ceil_avg = (W + k - 1) / k;
    int64_t slack = o - ceil_avg;
    if (slack <= 0) return o;
    if (slack < div) return o - 1;
    return o - slack / div;
}

/* slot() of Section 4.2.1 for integer losses: 2 + floor(log2 x) for x > 0. */
int32_t og_slot(int64_t x)
{
    if (x < 0) return 0;
    if (x == 0) return 1;
    int32_t fl = -1;
    while (x > 0) { fl++; x >>= 1; }
    return 2 + fl;
}

/* Order-independent digest of a partition: sum of mix64((v << 32) | P[v]). */
uint64_t og_digest(int32_t n, const int32_t *P)
{
    uint64_t d = 0;
    for (int32_t v = 0; v < n; v++)
        d += og_mix64(((uint64_t)(uint32_t)v << 32) | (uint32_t)P[v]);
    return d;
}

/* conn(v, p) for all parts p adjacent to v, accumulated into a dense array;
 * og_conn_clear resets exactly the entries og_conn_fill touched. */
static void og_conn_fill(const og_graph *g, const int32_t *P, int32_t v, int64_t *conn)
{
    for (int64_t e = g->xadj[v]; e < g->xadj[v + 1]; e++)
        conn[P[g->adjncy[e]]] += g->adjwgt[e];
}
static void og_conn_clear(const og_graph *g, const int32_t *P, int32_t v, int64_t *conn)
{
    for (int64_t e = g->xadj[v]; e < g->xadj[v + 1]; e++)
        conn[P[g->adjncy[e]]] = 0;
}

static void og_default_c(const og_params *prm, int32_t *cn, int32_t *cd)
{
    if (prm->c_den > 0) { *cn = prm->c_num; *cd = prm->c_den; return; }
    /* c = 0.25 at the finest level, 0.75 at every coarser level (Section 4.1.2) */
    if (prm->level == 0) { *cn = 1; *cd = 4; } else { *cn = 3; *cd = 4; }
}

/* ---- Jetlp (Algorithm 4) ------------------------------------------------
 * For every unlocked v: P_d = the most connected part other than P_s
 * (reading: ties -> smallest part id), F = conn(P_d) - conn(P_s). The first
 * filter admits v into X when F >= 0 or -F < floor(c * conn(v, P_s)).
 * The afterburner recomputes the gain F2 of each v in X against a
 * neighbourhood where every neighbour u that precedes v in ord (u in X with
 * a larger F, or equal F and smaller id) is assumed already in P_d(u).
 * Moves with F2 >= 0 form M. Outputs are per vertex; F = INT64_MIN marks
 * "no adjacent other part". Returns |M|; *nX_out = |X|. */
int32_t og_jetlp(const og_graph *g, const og_params *prm, const int32_t *P,
                 const uint8_t *locked, int32_t *pd, int64_t *F, int64_t *conn_s,
                 uint8_t *inX, int64_t *F2, uint8_t *move, int32_t *nX_out)
{
    int32_t n = g->n, k = prm->k, cn, cd;
    og_default_c(prm, &cn, &cd);
    int64_t *conn = (int64_t *)calloc((size_t)k, sizeof(int64_t));
    int32_t nX = 0, nM = 0;
    for (int32_t v = 0; v < n; v++) {
        pd[v] = P[v]; F[v] = INT64_MIN; conn_s[v] = 0; inX[v] = 0; F2[v] = 0; move[v] = 0;
        if (locked[v]) continue;
        og_conn_fill(g, P, v, conn);
        int32_t ps = P[v], best = -1;
        int64_t bestc = 0;
        for (int64_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
            int32_t p = P[g->adjncy[e]];
            if (p == ps || conn[p] <= 0) continue;
            if (best < 0 || conn[p] > bestc || (conn[p] == bestc && p < best)) { best = p; bestc = conn[p]; }
        }
        conn_s[v] = conn[ps];
        if (best >= 0) {
            pd[v] = best;
            F[v] = bestc - conn[ps];
            int64_t thr = ((int64_t)cn * conn[ps]) / cd; /* floor: both operands >= 0 */
            if (F[v] >= 0 || -F[v] < thr) { inX[v] = 1; nX++; }
        }
        og_conn_clear(g, P, v, conn);
    }
    for (int32_t v = 0; v < n; v++) {
        if (!inX[v]) continue;
        if (prm->flags & OG_F_NO_AFTERBURNER) { move[v] = 1; nM++; continue; }
        int64_t f2 = 0;
        for (int64_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
            int32_t u = g->adjncy[e];
            int32_t q = P[u];
            if (inX[u] && (F[u] > F[v] || (F[u] == F[v] && u < v))) q = pd[u];
            if (q == pd[v]) f2 += g->adjwgt[e];
            else if (q == P[v]) f2 -= g->adjwgt[e];
        }
        F2[v] = f2;
        if (f2 >= 0) { move[v] = 1; nM++; }
    }
    free(conn);
    if (nX_out) *nX_out = nX;
    return nM;
}

/* ---- rebalancing (Algorithm 5 and Jetrs) ------------------------------- */
typedef struct { int32_t slot, v; } og_key;
static int og_key_cmp(const void *a, const void *b)
{
    const og_key *x = (const og_key *)a, *y = (const og_key *)b;
    if (x->slot != y->slot) return x->slot < y->slot ? -1 : 1;
    return x->v < y->v ? -1 : (x->v > y->v);
}

/* One rebalancing step (kind OG_RW or OG_RS) against partition P with
 * iteration index t. dest[v] = destination or -1. Optional outputs:
 * loss[v] (INT64_MIN if not eligible), slot[v] (-1 if not eligible),
 * cand_dest[v] (Jetrw destination before eviction, -1 if not eligible).
 * Returns |M|; *ncand = number of eligible vertices. */
int32_t og_rebalance(const og_graph *g, const og_params *prm, const int32_t *P, int32_t kind,
                     int32_t t, int32_t *dest, int64_t *loss_out, int32_t *slot_out,
                     int32_t *cand_dest_out, int32_t *ncand_out)
{
    int32_t n = g->n, k = prm->k;
    int64_t W = og_total_weight(g);
    int64_t *w = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    og_part_weights(g, P, k, w);
    int64_t o = og_limit(W, k, prm->lambda_ppm);
    int64_t sigma = og_sigma(W, k, o, prm->deadzone_div > 0 ? prm->deadzone_div : 10);
    uint8_t *inA = (uint8_t *)calloc((size_t)k, 1), *inB = (uint8_t *)calloc((size_t)k, 1);
    int32_t *Blist = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
    int32_t nB = 0;
    for (int32_t p = 0; p < k; p++) {
        inA[p] = w[p] > o;
        inB[p] = w[p] <= sigma;
        if (inB[p]) Blist[nB++] = p;
    }
    int64_t *conn = (int64_t *)calloc((size_t)k, sizeof(int64_t));
    int64_t *loss = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t *slot = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *cdst = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    uint64_t hseed = og_mix64(prm->seed ^ (((uint64_t)(uint32_t)prm->level << 32) + (uint64_t)(uint32_t)t));
    int32_t ncand = 0;
    for (int32_t v = 0; v < n; v++) {
        dest[v] = -1; loss[v] = INT64_MIN; slot[v] = -1; cdst[v] = -1;
        int32_t ps = P[v];
        if (!inA[ps]) continue;
        /* heavy-vertex restriction: vw <= 1.5 (w(p_a) - W/k) */
        if (2 * (int64_t)k * g->vwgt[v] > 3 * ((int64_t)k * w[ps] - W)) continue;
        ncand++;
        og_conn_fill(g, P, v, conn);
        if (kind == OG_RW) {
            int32_t best = -1;
            int64_t bestc = 0;
            for (int64_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
                int32_t p = P[g->adjncy[e]];
                if (!inB[p] || conn[p] <= 0) continue;
                if (best < 0 || conn[p] > bestc || (conn[p] == bestc && p < best)) { best = p; bestc = conn[p]; }
            }
            if (best < 0) {
                /* randomPart(B): counter hash of (seed, level, t, v) */
                uint64_t h = og_mix64(hseed ^ (uint64_t)(uint32_t)v);
                best = Blist[og_below(h, (uint64_t)nB)];
            }
            cdst[v] = best;
            loss[v] = conn[ps] - conn[best];
        } else {
            /* mean connectivity over the adjacent valid destinations (floor) */
            int64_t sum = 0, cnt = 0;
            for (int32_t i = 0; i < nB; i++)
                if (conn[Blist[i]] > 0) { sum += conn[Blist[i]]; cnt++; }
            int64_t mean = cnt ? sum / cnt : 0;
            loss[v] = conn[ps] - mean;
        }
        slot[v] = og_slot(loss[v]);
        og_conn_clear(g, P, v, conn);
    }
    /* eviction: per oversized part, walk L' = eligible vertices ordered by
     * (slot, vertex id); evict while the weight evicted so far < w(p) - o. */
    uint8_t *evicted = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    og_key *L = (og_key *)malloc(sizeof(og_key) * (size_t)(n > 0 ? n : 1));
    for (int32_t p = 0; p < k; p++) {
        if (!inA[p]) continue;
        int32_t len = 0;
        for (int32_t v = 0; v < n; v++)
            if (P[v] == p && slot[v] >= 0) { L[len].slot = slot[v]; L[len].v = v; len++; }
        qsort(L, (size_t)len, sizeof(og_key), og_key_cmp);
        int64_t need = w[p] - o, s = 0;
        for (int32_t i = 0; i < len; i++) {
            if (s >= need) break;
            evicted[L[i].v] = 1;
            s += g->vwgt[L[i].v];
        }
    }
    int32_t nM = 0;
    if (kind == OG_RW) {
        for (int32_t v = 0; v < n; v++)
            if (evicted[v]) { dest[v] = cdst[v]; nM++; }
    } else {
        /* cookie-cutter: B in ascending id with capacity sigma - w(b); the
         * evicted vertices in ascending id; each takes the destination whose
         * capacity interval holds the weight evicted before it. */
        int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nB > 0 ? nB : 1));
        int64_t acc = 0;
        for (int32_t i = 0; i < nB; i++) { start[i] = acc; acc += sigma - w[Blist[i]]; }
        int64_t total = acc, pos = 0;
        for (int32_t v = 0; v < n; v++) {
            if (!evicted[v]) continue;
            if (pos < total) {
                int32_t b = -1;
                for (int32_t i = 0; i < nB; i++)
                    if (start[i] <= pos && pos < start[i] + (sigma - w[Blist[i]])) { b = Blist[i]; break; }
                dest[v] = b;
                nM++;
            }
            pos += g->vwgt[v];
        }
        free(start);
    }
    if (loss_out) memcpy(loss_out, loss, sizeof(int64_t) * (size_t)n);
    if (slot_out) memcpy(slot_out, slot, sizeof(int32_t) * (size_t)n);
    if (cand_dest_out) memcpy(cand_dest_out, cdst, sizeof(int32_t) * (size_t)n);
    if (ncand_out) *ncand_out = ncand;
    free(w); free(inA); free(inB); free(Blist); free(conn); free(loss); free(slot); free(cdst);
    free(evicted); free(L);
    return nM;
}

/* ---- refinement loop (Algorithm 3) -------------------------------------
 * part: in P_0, out P_best. iter_part (optional): P_iter at exit.
 * Returns the number of iterations run; traces the first trace_cap. */
int32_t og_refine(const og_graph *g, const og_params *prm, int32_t *part, og_trace *trace,
                  int32_t trace_cap, int32_t *iter_part, int64_t *stats /* [4]: cut, maxw, balanced, o */)
{
    int32_t n = g->n, k = prm->k;
    int64_t W = og_total_weight(g);
    int64_t o = og_limit(W, k, prm->lambda_ppm);
    if (k == 1) {
        for (int32_t v = 0; v < n; v++) part[v] = 0;
        if (iter_part) for (int32_t v = 0; v < n; v++) iter_part[v] = 0;
        if (stats) { stats[0] = 0; stats[1] = W; stats[2] = 1; stats[3] = o; }
        return 0;
    }
    size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t *P = (int32_t *)malloc(sizeof(int32_t) * nn);
    int32_t *best = (int32_t *)malloc(sizeof(int32_t) * nn);
    int32_t *pd = (int32_t *)malloc(sizeof(int32_t) * nn);
    int32_t *dest = (int32_t *)malloc(sizeof(int32_t) * nn);
    int64_t *F = (int64_t *)malloc(sizeof(int64_t) * nn);
    int64_t *cs = (int64_t *)malloc(sizeof(int64_t) * nn);
    int64_t *F2 = (int64_t *)malloc(sizeof(int64_t) * nn);
    uint8_t *inX = (uint8_t *)malloc(nn), *move = (uint8_t *)malloc(nn);
    uint8_t *locked = (uint8_t *)calloc(nn, 1);
    int64_t *w = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    memcpy(P, part, sizeof(int32_t) * (size_t)n);
    memcpy(best, part, sizeof(int32_t) * (size_t)n);
    og_part_weights(g, P, k, w);
    int64_t cut = og_cut(g, P), maxw = og_max(w, k);
    int balanced = maxw <= o;
    int bal_best = balanced;
    int64_t cut_best = cut, maxw_best = maxw;
    int32_t stall = 0, wcount = 0, t = 0;
    int32_t limit = prm->stall_limit > 0 ? prm->stall_limit : 12;
    int32_t bmax = prm->bmax >= 0 ? prm->bmax : 2;
    int64_t pn = prm->phi_num > 0 ? prm->phi_num : 999, pdn = prm->phi_den > 0 ? prm->phi_den : 1000;
    while (stall < limit && (prm->max_iters <= 0 || t < prm->max_iters)) {
        /* reading: every iteration counts toward the stall limit; the events
         * below reset the counter. */
        stall++;
        int32_t kind, nX = 0, nM = 0;
        int64_t moved_w = 0;
        if (balanced) {
            kind = OG_LP;
            nM = og_jetlp(g, prm, P, locked, pd, F, cs, inX, F2, move, &nX);
            /* R <- vertices moved by this Jetlp; rebalancing leaves R alone */
            for (int32_t v = 0; v < n; v++) {
                locked[v] = (prm->flags & OG_F_NO_LOCKS) ? 0 : move[v];
                dest[v] = move[v] ? pd[v] : -1;
            }
            wcount = 0;
        } else if (wcount < bmax) {
            kind = OG_RW;
            nM = og_rebalance(g, prm, P, OG_RW, t, dest, NULL, NULL, NULL, &nX);
            wcount++;
        } else {
            kind = OG_RS;
            nM = og_rebalance(g, prm, P, OG_RS, t, dest, NULL, NULL, NULL, &nX);
            wcount++;
        }
        /* all moves are applied against the state at the start of the
         * iteration (synchronous update) */
        for (int32_t v = 0; v < n; v++)
            if (dest[v] >= 0) { moved_w += g->vwgt[v]; P[v] = dest[v]; }
        og_part_weights(g, P, k, w);
        cut = og_cut(g, P);
        maxw = og_max(w, k);
        balanced = maxw <= o;
        if (balanced) {
            if (!bal_best) {
                /* reading: a balanced partition always beats an imbalanced best */
                memcpy(best, P, sizeof(int32_t) * (size_t)n);
                bal_best = 1; cut_best = cut; maxw_best = maxw; stall = 0;
            } else if (cut < cut_best) {
                if (pdn * cut < pn * cut_best) stall = 0; /* cut < phi * cut_best */
                memcpy(best, P, sizeof(int32_t) * (size_t)n);
                cut_best = cut; maxw_best = maxw;
            }
        } else if (!bal_best && maxw < maxw_best) {
            memcpy(best, P, sizeof(int32_t) * (size_t)n);
            maxw_best = maxw; cut_best = cut; stall = 0;
        }
        if (trace && t < trace_cap) {
            og_trace *r = &trace[t];
            r->level = prm->level; r->t = t; r->kind = kind; r->nX = nX; r->nM = nM;
            r->stall = stall; r->wcount = wcount; r->balanced = balanced;
            r->moved_w = moved_w; r->cut = cut; r->maxw = maxw; r->best_cut = cut_best;
            r->digest = og_digest(n, P);
        }
        t++;
    }
    memcpy(part, best, sizeof(int32_t) * (size_t)n);
    if (iter_part) memcpy(iter_part, P, sizeof(int32_t) * (size_t)n);
    if (stats) {
        og_part_weights(g, best, k, w);
        stats[0] = cut_best; stats[1] = og_max(w, k); stats[2] = og_max(w, k) <= o; stats[3] = o;
    }
    free(P); free(best); free(pd); free(dest); free(F); free(cs); free(F2);
    free(inX); free(move); free(locked); free(w);
    return t;
}

/* ---- two-hop matching (Section 3.1) --------------------------------------
 * reading: after the heavy-edge rounds, while more than a quarter of the
 * vertices is unmatched, three passes add matches between vertices two hops
 * apart, each pass only if the previous one left more than n/4 unmatched:
 *   leaves     unmatched vertices of degree 1, keyed by their neighbour;
 *   twins      unmatched vertices of 1 to 64 entries keyed by their
 *              neighbourhood: the hash mix64(h ^ mix64(deg)) >> 1 of
 *              h = sum over neighbours u of mix64(u + 1) (mod 2^64)
 *              (twins are relatives, two hops apart, so isolated vertices
 *              never pair);
 *   relatives  unmatched vertices of 1 to 64 entries keyed by their
 *              matchmaker, the smallest-id neighbour that is already matched
 *              and has at most 1024 entries (hubs never act as matchmakers).
 * Vertices with equal keys are matched in ascending id order, first with
 * second, third with fourth, and so on. */
#define OG_TWO_HOP_MM_MAXDEG 1024
#define OG_TWO_HOP_MAXDEG 64

typedef struct { uint64_t key; int32_t v; } og_kv;
static int og_kv_cmp(const void *a, const void *b)
{
    const og_kv *x = (const og_kv *)a, *y = (const og_kv *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->v < y->v ? -1 : (x->v > y->v);
}

static int32_t og_unmatched(const int32_t *match, int32_t n)
{
    int32_t c = 0;
    for (int32_t v = 0; v < n; v++) c += match[v] < 0;
    return c;
}

/* pairs vertices of equal key (candidates only) in ascending id order */
static void og_pair_by_key(int32_t *match, og_kv *kv, int32_t m)
{
    qsort(kv, (size_t)m, sizeof(og_kv), og_kv_cmp);
    int32_t i = 0;
    while (i < m) {
        int32_t j = i;
        while (j < m && kv[j].key == kv[i].key) j++;
        for (int32_t a = i; a + 1 < j; a += 2) {
            match[kv[a].v] = kv[a + 1].v;
            match[kv[a + 1].v] = kv[a].v;
        }
        i = j;
    }
}

static void og_two_hop(const og_graph *g, int32_t *match)
{
    int32_t n = g->n;
    if (n == 0) return;
    og_kv *kv = (og_kv *)malloc(sizeof(og_kv) * (size_t)n);
    for (int pass = 0; pass < 3; pass++) {
        if (4 * (int64_t)og_unmatched(match, n) <= (int64_t)n) break;
        int32_t m = 0;
        for (int32_t v = 0; v < n; v++) {
            if (match[v] >= 0) continue;
            int64_t deg = g->xadj[v + 1] - g->xadj[v];
            if (deg < 1 || deg > OG_TWO_HOP_MAXDEG) continue;
            if (pass == 0) {
                if (deg != 1) continue;
                kv[m].key = (uint64_t)(uint32_t)g->adjncy[g->xadj[v]];
            } else if (pass == 1) {
                uint64_t h = 0;
                for (int64_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) h += og_mix64((uint64_t)(uint32_t)g->adjncy[e] + 1);
                kv[m].key = og_mix64(h ^ og_mix64((uint64_t)deg)) >> 1;
            } else {
                int32_t mm = -1;
                for (int64_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
                    int32_t u = g->adjncy[e];
                    if (match[u] < 0 || g->xadj[u + 1] - g->xadj[u] > OG_TWO_HOP_MM_MAXDEG) continue;
                    if (mm < 0 || u < mm) mm = u;
                }
                if (mm < 0) continue;
                kv[m].key = (uint64_t)(uint32_t)mm;
            }
            kv[m].v = v;
            m++;
        }
        og_pair_by_key(match, kv, m);
    }
    free(kv);
}

/* ---- multilevel scaffold: heavy-edge matching + contraction ------------
 * reading (the paper names heavy-edge matching but not its tie rules):
 * rounds of mutual proposals. Each unmatched vertex proposes to the
 * unmatched neighbour across its heaviest edge; ties go to the smaller
 * edge hash mix64(hseed ^ (min << 32 | max)), then to the smaller id.
 * Mutual proposals match. Rounds stop after 16, or once a round matches
 * fewer than 1% of the vertices. hseed = stream(seed, level). With
 * two_hop, two-hop matching (above) then adds pairs when many vertices
 * stay unmatched.
 * Coarse ids: vertices that are unmatched or the smaller end of their pair
 * are leaders, numbered in vertex order. Returns the coarse vertex count. */
int32_t og_hem_map(const og_graph *g, int32_t level, uint64_t seed, int32_t two_hop, int32_t *map)
{
    int32_t n = g->n;
    size_t nn = (size_t)(n > 0 ? n : 1);
    int32_t *match = (int32_t *)malloc(sizeof(int32_t) * nn);
    int32_t *prop = (int32_t *)malloc(sizeof(int32_t) * nn);
    uint64_t hseed = og_stream(seed, (uint64_t)(uint32_t)level);
    for (int32_t v = 0; v < n; v++) match[v] = -1;
    for (int32_t round = 0; round < 16; round++) {
        for (int32_t v = 0; v < n; v++) {
            prop[v] = -1;
            if (match[v] >= 0) continue;
            int32_t bu = -1; int64_t bw = 0; uint64_t bh = 0;
            for (int64_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
                int32_t u = g->adjncy[e];
                if (match[u] >= 0) continue;
                int64_t wt = g->adjwgt[e];
                uint32_t a = (uint32_t)(u < v ? u : v), b = (uint32_t)(u < v ? v : u);
                uint64_t h = og_mix64(hseed ^ (((uint64_t)a << 32) | b));
                if (bu < 0 || wt > bw || (wt == bw && (h < bh || (h == bh && u < bu)))) {
                    bu = u; bw = wt; bh = h;
                }
            }
            prop[v] = bu;
        }
        int64_t newly = 0;
        for (int32_t v = 0; v < n; v++) {
            int32_t u = prop[v];
            if (u > v && prop[u] == v) { match[v] = u; match[u] = v; newly += 2; }
        }
        if (newly == 0 || newly * 100 < (int64_t)n) break;
    }
    if (two_hop) og_two_hop(g, match);
    int32_t nc = 0;
    for (int32_t v = 0; v < n; v++)
        if (match[v] < 0 || v < match[v]) map[v] = nc++;
    for (int32_t v = 0; v < n; v++)
        if (match[v] >= 0 && match[v] < v) map[v] = map[match[v]];
    free(match); free(prop);
    return nc;
}

static int og_int_cmp(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return x < y ? -1 : (x > y);
}

/* Contraction (Algorithm 2 computes the same thing with per-row hashing):
 * coarse vertex weight = sum of member weights; coarse edge (a, b), a != b,
 * carries the summed weight of all fine edges between members of a and b.
 * Coarse rows come out sorted by neighbour id. Caller frees the arrays. */
void og_contract(const og_graph *g, const int32_t *map, int32_t nc, int64_t **cxadj,
                 int32_t **cadj, int32_t **cvw, int32_t **cew)
{
    int32_t n = g->n;
    size_t ncc = (size_t)(nc > 0 ? nc : 1);
    int32_t *vw = (int32_t *)calloc(ncc, sizeof(int32_t));
    /* member lists of each coarse vertex */
    int64_t *mstart = (int64_t *)calloc(ncc + 1, sizeof(int64_t));
    int32_t *members = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t v = 0; v < n; v++) { mstart[map[v] + 1]++; vw[map[v]] += g->vwgt[v]; }
    for (int32_t c = 0; c < nc; c++) mstart[c + 1] += mstart[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ncc);
    for (int32_t c = 0; c < nc; c++) fill[c] = mstart[c];
    for (int32_t v = 0; v < n; v++) members[fill[map[v]]++] = v;
    /* dense accumulator over coarse neighbours */
    int64_t *acc = (int64_t *)calloc(ncc, sizeof(int64_t));
    int32_t *seen = (int32_t *)malloc(sizeof(int32_t) * ncc);
    for (int32_t c = 0; c < nc; c++) seen[c] = -1;
    int64_t cap = g->xadj[n] > 0 ? g->xadj[n] : 1;
    int32_t *adj = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    int32_t *ew = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    int32_t *row = (int32_t *)malloc(sizeof(int32_t) * ncc);
    int64_t *xadj = (int64_t *)calloc(ncc + 1, sizeof(int64_t));
    int64_t pos = 0;
    for (int32_t c = 0; c < nc; c++) {
        int32_t len = 0;
        for (int64_t i = mstart[c]; i < mstart[c + 1]; i++) {
            int32_t v = members[i];
            for (int64_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
                int32_t cu = map[g->adjncy[e]];
                if (cu == c) continue;
                if (seen[cu] != c) { seen[cu] = c; acc[cu] = 0; row[len++] = cu; }
                acc[cu] += g->adjwgt[e];
            }
        }
        qsort(row, (size_t)len, sizeof(int32_t), og_int_cmp);
        for (int32_t i = 0; i < len; i++) { adj[pos] = row[i]; ew[pos] = (int32_t)acc[row[i]]; pos++; }
        xadj[c + 1] = pos;
    }
    *cxadj = xadj; *cadj = adj; *cvw = vw; *cew = ew;
    free(mstart); free(members); free(fill); free(acc); free(seen); free(row);
}

void og_free(void *p) { free(p); }

/* ---- graph-growing start of the coarsest graph ---------------------------
 * Not from the paper, whose coarsest partition comes from Metis (Section 3):
 * every connected component is searched breadth-first from its smallest
 * vertex id; vertices are ordered by (that id, distance from it, own id) and
 * the order is cut into k consecutive runs of equal vertex weight: a vertex
 * whose predecessors in the order weigh b goes to part floor(b k / W), W the
 * total vertex weight (W = 0: part 0). */
typedef struct { int32_t root, dist, v; } og_bkey;

static int og_bkey_cmp(const void *pa, const void *pb)
{
    const og_bkey *a = (const og_bkey *)pa, *b = (const og_bkey *)pb;
    if (a->root != b->root) return a->root < b->root ? -1 : 1;
    if (a->dist != b->dist) return a->dist < b->dist ? -1 : 1;
    return (a->v > b->v) - (a->v < b->v);
}

void og_bfs_part(const og_graph *g, int32_t k, int32_t *part)
{
    const int32_t n = g->n;
    if (n <= 0) return;
    int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    og_bkey *order = (og_bkey *)malloc(sizeof(og_bkey) * (size_t)n);
    for (int32_t v = 0; v < n; v++) dist[v] = -1;
    for (int32_t r = 0; r < n; r++) {
        if (dist[r] >= 0) continue;
        int32_t head = 0, tail = 0;
        queue[tail++] = r;
        dist[r] = 0;
        while (head < tail) {
            const int32_t v = queue[head++];
            order[v].root = r;
            order[v].dist = dist[v];
            order[v].v = v;
            for (int64_t e = g->xadj[v]; e < g->xadj[v + 1]; e++) {
                const int32_t u = g->adjncy[e];
                if (dist[u] < 0) {
                    dist[u] = dist[v] + 1;
                    queue[tail++] = u;
                }
            }
        }
    }
    qsort(order, (size_t)n, sizeof(og_bkey), og_bkey_cmp);
    int64_t W = 0;
    for (int32_t v = 0; v < n; v++) W += g->vwgt ? g->vwgt[v] : 1;
    int64_t b = 0;
    for (int32_t i = 0; i < n; i++) {
        const int32_t v = order[i].v;
        part[v] = W > 0 ? (int32_t)(((unsigned __int128)(uint64_t)b * (uint64_t)k) / (uint64_t)W) : 0;
        b += g->vwgt ? g->vwgt[v] : 1;
    }
    free(dist);
    free(queue);
    free(order);
}

/* ---- multilevel template (Algorithm 1) ---------------------------------
 * Coarsen until n <= 8k (Section 3's target), or 64 levels. A matching that
 * would keep more than 90% of the vertices (or matches nothing) makes no
 * level: the current level is the coarsest;
 * seeded uniform random partition of the coarsest graph,
 * P[v] = floor(stream(mix64(seed ^ 1), v) * k / 2^64), or with
 * OG_F_BFS_START the graph-growing start og_bfs_part; refine it; then
 * project (P_i[v] = P_{i+1}[map_i[v]]) and refine each finer level.
 * Level numbers: 0 = input graph. Returns the number of levels (>= 1).
 * level_sizes (optional, [64]) receives n of each level. */
int32_t og_partition(const og_graph *g, const og_params *prm, int32_t *part, og_trace *trace,
                     int32_t trace_cap, int32_t *ntrace, int32_t *level_sizes, int64_t *stats)
{
    enum { MAXL = 64 };
    og_graph G[MAXL];
    int32_t *maps[MAXL];
    int32_t nl = 1;
    int32_t k = prm->k;
    G[0] = *g;
    while (nl < MAXL && G[nl - 1].n > 8 * (int64_t)k) {
        const og_graph *f = &G[nl - 1];
        int32_t *map = (int32_t *)malloc(sizeof(int32_t) * (size_t)(f->n > 0 ? f->n : 1));
        int32_t nc = og_hem_map(f, nl - 1, prm->seed, (prm->flags & OG_F_TWO_HOP) != 0, map);
        if (nc == f->n || 10 * (int64_t)nc > 9 * (int64_t)f->n) { free(map); break; }
        int64_t *cx; int32_t *ca, *cv, *cw;
        og_contract(f, map, nc, &cx, &ca, &cv, &cw);
        maps[nl - 1] = map;
        G[nl].n = nc; G[nl].xadj = cx; G[nl].adjncy = ca; G[nl].vwgt = cv; G[nl].adjwgt = cw;
        nl++;
    }
    if (level_sizes) for (int32_t i = 0; i < nl; i++) level_sizes[i] = G[i].n;
    int32_t l = nl - 1;
    int32_t *P = (int32_t *)malloc(sizeof(int32_t) * (size_t)(G[l].n > 0 ? G[l].n : 1));
    if (prm->flags & OG_F_BFS_START) {
        og_bfs_part(&G[l], k, P);
    } else {
        uint64_t s_init = og_mix64(prm->seed ^ 1ULL);
        for (int32_t v = 0; v < G[l].n; v++) P[v] = (int32_t)og_below(og_stream(s_init, (uint64_t)v), (uint64_t)k);
    }
    int32_t tr = 0;
    for (int32_t i = l; i >= 0; i--) {
        if (i < l) {
            int32_t *Pf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(G[i].n > 0 ? G[i].n : 1));
            for (int32_t v = 0; v < G[i].n; v++) Pf[v] = P[maps[i][v]];
            free(P);
            P = Pf;
        }
        og_params q = *prm;
        q.level = i;
        int32_t it = og_refine(&G[i], &q, P, trace ? trace + tr : NULL, trace ? trace_cap - tr : 0, NULL,
                               i == 0 ? stats : NULL);
        tr += it < (trace_cap - tr) ? it : (trace_cap - tr);
    }
    memcpy(part, P, sizeof(int32_t) * (size_t)g->n);
    if (ntrace) *ntrace = tr;
    free(P);
    for (int32_t i = 1; i < nl; i++) {
        free((void *)G[i].xadj); free((void *)G[i].adjncy); free((void *)G[i].vwgt); free((void *)G[i].adjwgt);
        free(maps[i - 1]);
    }
    return nl;
}
