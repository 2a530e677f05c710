/*
 * jet.h -- C ABI of the MI355X (gfx950) Jet graph-partition refinement library.
 *
 * Implements the refinement pass of Jet (Gilbert, Madduri, Boman,
 * Rajamanickam, "Jet: Multilevel Graph Partitioning on Graphics Processing
 * Units"): part connectivity and gain, the Jetlp candidate filter and the
 * afterburner (Section 4.1, Algorithm 4), synchronous move application with
 * cut and part-weight updates, the refinement loop with best tracking
 * (Algorithm 3) and weak / strong rebalancing through loss slots
 * (Section 4.2, Algorithm 5); and, as the surrounding multilevel scaffold,
 * heavy-edge matching, contraction (Algorithm 2) and projection
 * (Algorithm 1).
 *
 * Conventions
 *  - Every pointer inside jet_csr, and `part`, are DEVICE pointers unless a
 *    comment says (host). The caller owns them; the library never frees them.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream). All
 *    device work is ordered on it: the coarsening forks the hub rows'
 *    contraction onto a second stream of the context, which waits on
 *    `stream` and is joined back to it within the call. Calls return after
 *    the stream has finished the call's work (they synchronise it), except
 *    jet_refine with JET_F_ASYNC.
 *  - Status codes are returned as int; no exception crosses the ABI. On an
 *    error detected before any device work, `part` is untouched; after device
 *    work has started, `part` is unspecified.
 *  - Graph (Section 2.1): undirected, no self-loops, no parallel edges; each
 *    edge is stored in both rows. Vertex and edge weights are positive
 *    integers. Arithmetic is integer only: int32 weights, int64 cuts, gains
 *    and part weights. Results are deterministic and independent of thread
 *    scheduling: ties break by part id or vertex id, never by atomic order.
 *  - Limits: n < 2^31; 1 <= k <= 16384; the total vertex weight below 2^31
 *    and every vertex's weighted degree (sum of its edge weights) below 2^31
 *    (else JET_EOVERFLOW): connectivities, gains and losses, which that degree
 *    bounds, are int32, while cuts and part weights are int64. Multilevel
 *    calls (jet_coarsen, jet_partition, serving jobs) also need the total edge
 *    weight (summed over both directions) below 2^31, because coarse edge
 *    weights are sums of fine ones and are stored as int32.
 *  - One context per host thread, or external locking.
 */
#ifndef JET_H
#define JET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define JET_OK         0
#define JET_EINVAL    (-1) /* bad parameter (k < 1, lambda < 0, c_den < 0, NULL pointer, ...) */
#define JET_EGRAPH    (-2) /* malformed CSR (checked cheaply always, fully with JET_F_VALIDATE) */
#define JET_EPART     (-3) /* a part id outside [0, k) */
#define JET_EOVERFLOW (-4) /* a weight total or a weighted degree >= 2^31 (see Limits) */
#define JET_ENOMEM    (-5) /* device or host allocation failed */
#define JET_EHIP      (-6) /* HIP runtime error; jet_last_hip_error() has the code */
#define JET_EAGAIN    (-7) /* serving: queue full, or the job is not done yet */
#define JET_ELIMIT    (-8) /* outside a documented size limit (e.g. k > 16384) */

/* ---- flags ------------------------------------------------------------- */
#define JET_F_VALIDATE    0x1u  /* full CSR check: range, self-loops, symmetry, duplicates */
#define JET_F_RETURN_ITER 0x2u  /* return P_iter (state after the last iteration) instead of P_best */
#define JET_F_PROFILE     0x4u  /* time the connectivity/gain passes (see jet_stats.ms_gain) */
/* Jetlp ablations (Section 7.1, Component Effectiveness, Table lp_versions):
 * without locks, a vertex moved by one Jetlp may move again in the next;
 * without the afterburner, every vertex of X moves (F2 is reported as 0).
 * The paper's "weak afterburner" admits only moves with F >= 0: set
 * c_num = 0, c_den = 1. The baseline synchronous LP is all three. */
#define JET_F_LP_NO_LOCKS       0x8u
#define JET_F_LP_NO_AFTERBURNER 0x10u
/* Coarsening (jet_coarsen, jet_partition, serving jobs): after heavy-edge
 * matching, while more than a quarter of the vertices is unmatched, add
 * two-hop matches (Section 3.1): leaves (one entry, same neighbour), twins
 * (1 to 64 entries, same neighbourhood hash), relatives (1 to 64 entries,
 * same matchmaker: the smallest-id matched neighbour of at most 1024
 * entries); equal keys pair in ascending id order. */
#define JET_F_TWO_HOP           0x20u
/* Multilevel partition (jet_partition, serving jobs): start the coarsest
 * graph from jet_bfs_start's graph-growing partition instead of the seeded
 * random one. */
#define JET_F_BFS_START         0x40u
/* jet_refine only: return without waiting for the refinement. The call still
 * waits once for its set-up (checks, degree classes, which size the
 * launches); it then enqueues max_iters iterations (max_iters > 0 is
 * required; the device-side controller ends the loop, and iterations past
 * the end exit at once), the result copies and a host function that fills
 * `stats` and the trace (count, total, records) when the stream reaches it.
 * `part`, part_weights_out, stats and the trace are valid once the stream
 * has completed (hipStreamSynchronize on it); stats' ms_* fields are 0. The
 * context must not be used again before that. JET_EINVAL with
 * max_iters <= 0 or JET_F_PROFILE, and on every other entry point. */
#define JET_F_ASYNC             0x80u
/* Single-graph refinement (jet_refine, jet_partition, steps, serving jobs on
 * their own lane; batches ignore it): keep Section 4.3's persistent
 * vertex-part connectivity structure instead of rebuilding connectivity
 * in LDS on every pass. Row v owns min(k, deg v) slots of (part, count),
 * hashed by part and sized a little above the parts v touches; after each
 * iteration the moves update the rows of their neighbours (Algorithm 6:
 * decrement the source part, then increment the destination part,
 * inserting it; a row without a free slot is rebuilt larger), or, when more
 * than a tenth of the vertices moved, every row is rebuilt. Gains and
 * losses then scan rows. Results are identical to the default (maxima are
 * taken on (count, part) keys); only speed and memory differ:
 * 8 (n + 1) + 8 sum_v min(k, deg v) + 12 n bytes. */
#define JET_F_CONN_TABLE        0x100u

typedef struct jet_context jet_context;
typedef struct jet_hierarchy jet_hierarchy;

/* Graph in CSR form (Section 2.1). Device pointers. */
typedef struct {
    int32_t n;              /* number of vertices */
    int32_t reserved;
    int64_t nnz;            /* = xadj[n] = 2m (every edge stored in both rows) */
    const int64_t *xadj;    /* [n+1], xadj[0] = 0, non-decreasing */
    const int32_t *adjncy;  /* [nnz], neighbour ids in [0, n) */
    const int32_t *vwgt;    /* [n] >= 1, or NULL for unit vertex weights */
    const int32_t *adjwgt;  /* [nnz] >= 1, symmetric, or NULL for unit edge weights */
} jet_csr;

/* Refinement parameters. Zero-initialise, set k and lambda_ppm, keep the
 * defaults by leaving the rest 0. */
typedef struct {
    int32_t k;                    /* number of parts, >= 1 */
    int32_t lambda_ppm;           /* imbalance lambda * 1e6 (3% = 30000); balance limit
                                     o = floor(W (1e6 + lambda_ppm) / (k 1e6)) */
    int32_t c_num, c_den;         /* first-filter ratio c of eq. gainconn_filter; c_den = 0 ->
                                     1/4 at level 0 and 3/4 at coarser levels (Section 4.1.2) */
    int32_t phi_num, phi_den;     /* loop tolerance phi of Algorithm 3; 0 -> 999/1000 */
    int32_t stall_limit;          /* iterations without a new best before stopping; 0 -> 12 */
    int32_t weak_rebalance_iters; /* Jetrw iterations before Jetrs (b_max); -1 -> 0, 0 -> 2 */
    int32_t deadzone_div;         /* sigma rule divisor; 0 -> 10 (see jet_refine) */
    int32_t level;                /* hierarchy level of the graph (0 = finest): selects the
                                     default c and seeds the random destination hash */
    int32_t max_iters;            /* safety cap on iterations, 0 = none */
    uint32_t flags;               /* JET_F_* */
    uint64_t seed;                /* seed of every random choice (SplitMix64) */
} jet_params;

/* Results of a call (host). */
typedef struct {
    int64_t cut;             /* cut of the returned partition */
    int64_t max_part_weight; /* max part weight of the returned partition */
    int64_t o;               /* balance limit */
    int64_t sigma;           /* deadzone bound */
    int64_t total_weight;    /* W */
    int32_t balanced;        /* returned partition satisfies max part weight <= o */
    int32_t iters;           /* refinement iterations (summed over levels for jet_partition) */
    int32_t lp_iters, rw_iters, rs_iters;
    int32_t levels;          /* hierarchy levels (jet_partition), 1 for jet_refine */
    float ms_total;          /* device time of the call (hipEvents) */
    float ms_refine;         /* device time spent in refinement iterations */
    float ms_coarsen;        /* device time spent coarsening (jet_partition) */
    float ms_init;           /* device time of per-level set-up (binning, cut, weights) */
    /* With JET_F_PROFILE, for the Jetlp iterations of the finest level (level
     * 0): summed device time of the connectivity/gain passes (hipEvents on
     * the call's stream around each pass), their count, the CSR entries and
     * unlocked rows they read and the vertices they visited. */
    float ms_gain;
    int32_t gain_passes;
    int64_t gain_entries, gain_rows, gain_vertices;
    /* jet_refine_batch: the autotuner's choice for the batch (how waves walk
     * the vertex lists: 0 = static stretches, else work-queue tiles of that
     * many visits of a wave; small-row group width, 4 or 8 lanes). */
    int32_t batch_tile, batch_group;
} jet_stats;

/* One record per refinement iteration (written when a trace is passed). */
typedef struct {
    int32_t level, t, kind;  /* kind: 1 Jetlp, 2 Jetrw, 3 Jetrs */
    int32_t nX;              /* Jetlp: |X|; rebalancing: number of eligible vertices */
    int32_t nM;              /* moves applied */
    int32_t stall, wcount, balanced;
    int64_t moved_w;         /* total weight of the moved vertices */
    int64_t cut, maxw;       /* of P_iter after the iteration */
    int64_t best_cut;        /* cut of P_best after the iteration */
    uint64_t digest;         /* sum over v of mix64((v << 32) | P_iter[v]) mod 2^64 */
} jet_trace_rec;

typedef struct {
    jet_trace_rec *recs;     /* (host) capacity `cap`; NULL = no trace */
    int32_t cap;
    int32_t count;           /* out: records written (<= cap) */
    int32_t total;           /* out: iterations run (may exceed cap) */
    int32_t reserved;
} jet_trace;

/* ---- context ----------------------------------------------------------- */
/* Creates a context bound to HIP device `device`. It owns the workspace pool
 * (grown on demand, reused across calls) and small pinned host buffers. */
int  jet_context_create(jet_context **ctx, int device);
void jet_context_destroy(jet_context *ctx);
const char *jet_strerror(int status);
int  jet_last_hip_error(const jet_context *ctx);

/* ---- refinement (Algorithm 3 with Algorithms 4 and 5) -------------------
 * Refines `part` (int32[n], device, in: P_0, out: P_best) of graph `g` into
 * k parts under balance lambda:
 *   - while balanced (max part weight <= o): a Jetlp iteration. For each
 *     unlocked v with another adjacent part: P_d = most connected other part
 *     (ties -> smallest id), F = conn(P_d) - conn(P_s); X = {F >= 0 or
 *     -F < floor(c conn(P_s))}; afterburner gain F2 over the ord-merged
 *     neighbourhood; M = {v in X : F2 >= 0}; the vertices of M are locked
 *     for the next Jetlp (Section 4.1.3).
 *   - else weak (Jetrw, first b_max iterations after a Jetlp) or strong
 *     (Jetrs) rebalancing: oversized parts A = {w > o}, valid destinations
 *     B = {w <= sigma}, sigma = o if slack = o - ceil(W/k) <= 0, o - 1 if
 *     slack < deadzone_div, else o - floor(slack / deadzone_div); eligible
 *     vertices 2k vw <= 3(k w(p) - W); loss slot 0 / 1 / 2 + floor(log2);
 *     per part, evict in (slot, vertex id) order while the weight already
 *     evicted is below w(p) - o. Jetrw sends each evicted vertex to its best
 *     connected B part (or B[floor(h * |B| / 2^64)] with
 *     h = mix64(mix64(seed ^ (level 2^32 + t)) ^ v) when it touches none);
 *     Jetrs overlays the evicted vertices, in id order, onto B's capacities
 *     sigma - w(b) in id order.
 *   - moves are applied simultaneously; the best balanced partition (or,
 *     while none is balanced, the least oversized) is kept; the loop stops
 *     after stall_limit iterations without a new best, where a new balanced
 *     best only restarts the count if cut < phi * best cut.
 * part_weights_out: optional device int64[k], weights of the returned
 * partition. stats (host, optional), trace (host, optional).
 * Errors: JET_EINVAL, JET_EGRAPH, JET_EPART, JET_EOVERFLOW, JET_ELIMIT,
 * JET_ENOMEM, JET_EHIP. */
int jet_refine(jet_context *ctx, const jet_csr *g, const jet_params *params, int32_t *part,
               int64_t *part_weights_out, jet_stats *stats, jet_trace *trace, void *stream);

/* ---- refinement without allocation ----------------------------------------
 * For callers that cannot allocate device memory during the call (code
 * running under stream capture of their own, tight serving loops, harnesses
 * that forbid hipMalloc): jet_refine with the same arguments, results, trace
 * and errors, whose workspace (per-vertex state, class lists, counters,
 * controller, histograms, tile sums, long-row chunk tables, trace staging)
 * is carved from one static device array of JET_NOALLOC_SCRATCH_BYTES per
 * GPU instead of the context's pool. The array is part of the library's
 * code object: every GPU the library runs on holds it until the process
 * ends. The call itself allocates nothing (no hipMalloc / hipFree, no host
 * or pinned allocation, no graph instantiation: iterations are launched
 * directly); the context must come from jet_context_create, which looks the
 * array up once per device.
 * Limits and restrictions: the workspace of (n, nnz, k, trace capacity) must
 * fit the array (about 33 bytes per vertex plus per-part, per-tile and
 * long-row terms; JET_ELIMIT before any device work otherwise, `part`
 * untouched); k >= 2 (JET_EINVAL for k = 1, answered by jet_refine);
 * JET_F_VALIDATE and JET_F_PROFILE are rejected (JET_EINVAL).
 * All calls on one GPU share its array, which keeps the previous call's
 * contents (every call initialises what it reads): calls that overlap in
 * time on one GPU, from any context or thread, race and must be serialised
 * by the caller. */
#define JET_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int jet_refine_noalloc(jet_context *ctx, const jet_csr *g, const jet_params *params, int32_t *part,
                       int64_t *part_weights_out, jet_stats *stats, jet_trace *trace, void *stream);

/* ---- batched refinement ---------------------------------------------------
 * Refines `count` independent graphs in one launch sequence: the graphs are
 * laid out as one block-diagonal union (graph i's vertices, parts and
 * selection tiles follow graph i-1's) and every iteration's kernels serve all
 * graphs at once, each graph with its own controller, so each runs exactly
 * the iterations it would run alone (Algorithm 3 applied per graph; no edge
 * joins two graphs, so no connectivity, gain or loss mixes them). Graph i's
 * result equals jet_refine(graphs[i], params[i], parts[i]) bit for bit,
 * trace included.
 *   graphs:  host array [count] of CSRs whose arrays are device pointers
 *   params:  host array [count]; per graph k, lambda, c, phi, stall limit,
 *            b_max, deadzone, level, seed, JET_F_VALIDATE, JET_F_RETURN_ITER
 *            (JET_F_PROFILE is ignored)
 *   parts:   host array [count] of device int32[n_i] (in: P_0, out: P_best)
 *   stats:   host array [count] or NULL (ms_* fields are the whole batch's)
 *   traces:  host array [count] or NULL; each with its own host buffer
 * Graphs with k = 1 or n = 0 are answered directly (all vertices in part 0).
 * Limits: the union must stay below 2^31 vertices and parts. Errors as for
 * jet_refine; the first invalid graph stops the call before any refinement
 * (parts are then unchanged, except that graphs answered directly may
 * already be written). */
int jet_refine_batch(jet_context *ctx, int32_t count, const jet_csr *graphs, const jet_params *params,
                     int32_t *const *parts, jet_stats *stats, jet_trace *traces, void *stream);

/* ---- single-step entry points (for step-level checks) --------------------
 * One Jetlp step (Algorithm 4) against `part` with lock flags `locked`
 * (device u8[n], nonzero = locked). Outputs (device, [n] each): pd (P_d, or
 * P_s when v has no other adjacent part or is locked), F (int64, INT64_MIN
 * when undefined), conn_s (int64, 0 when locked), inX (u8), F2 (int64, 0
 * outside X), move (u8). */
int jet_lp_step(jet_context *ctx, const jet_csr *g, const jet_params *params, const int32_t *part,
                const uint8_t *locked, int32_t *pd, int64_t *F, int64_t *conn_s, uint8_t *inX,
                int64_t *F2, uint8_t *move, void *stream);

/* One rebalancing step (kind 2 = Jetrw, 3 = Jetrs) at iteration index t.
 * Outputs (device, [n]): dest (destination or -1), loss (int64, INT64_MIN
 * when not eligible), slot (int32, -1 when not eligible). */
int jet_rebalance_step(jet_context *ctx, const jet_csr *g, const jet_params *params,
                       const int32_t *part, int32_t kind, int32_t t, int32_t *dest, int64_t *loss,
                       int32_t *slot, void *stream);

/* ---- multilevel scaffold (Algorithms 1 and 2) ---------------------------
 * jet_coarsen builds the hierarchy G_0 = g, G_1, ... by heavy-edge matching
 * (rounds of mutual proposals: heaviest edge to an unmatched neighbour, ties
 * to the smaller mix64(stream(seed, level) ^ (min << 32 | max)), then the
 * smaller id; at most 16 rounds, stopping when a round matches < 1% of the
 * vertices) and contraction (coarse ids = matched pairs and singletons
 * numbered by their smaller member; coarse edge weights summed; no
 * self-loops). Coarsening stops when n <= 8k, at 64 levels, or when a
 * matching would keep more than 90% of the vertices (that matching makes no
 * level; the current one is the coarsest). The hierarchy lives in device memory
 * owned by the library until jet_hierarchy_free. Rows of coarse graphs are
 * not sorted. */
int jet_coarsen(jet_context *ctx, const jet_csr *g, const jet_params *params, jet_hierarchy **h,
                void *stream);
int jet_hierarchy_levels(const jet_hierarchy *h);
/* view: device CSR of level `level` (level 0 = the input graph); map: device
 * int32[n_level] mapping level -> level+1 vertex (NULL for the coarsest). */
int jet_hierarchy_level(const jet_hierarchy *h, int level, jet_csr *view, const int32_t **map);
void jet_hierarchy_free(jet_hierarchy *h);

/* Full multilevel partition (Algorithm 1): coarsen, seeded uniform random
 * partition of the coarsest graph P[v] = floor(stream(mix64(seed ^ 1), v) k
 * / 2^64) (with JET_F_BFS_START: jet_bfs_start's partition), refine it, then
 * project and refine every finer level (c = 3/4
 * above level 0, 1/4 at level 0 unless params sets c). part_out: device
 * int32[n]. The trace, if given, concatenates the levels' records. */
int jet_partition(jet_context *ctx, const jet_csr *g, const jet_params *params, int32_t *part_out,
                  jet_stats *stats, jet_trace *trace, void *stream);

/* Graph-growing start (the paper takes its coarsest partition from Metis and
 * leaves a GPU initial partitioner to future work, Section 3): every
 * connected component is grown breadth-first from its smallest vertex id;
 * vertices are ordered by (that id, BFS distance from it, own id), and the
 * order is cut into k runs of equal vertex weight: the vertex whose
 * predecessors in the order weigh b gets part floor(b k / W), W the total
 * vertex weight. Deterministic (no seed). part: device int32[n], written.
 * Returns JET_EINVAL (NULL pointers, k < 1), JET_ELIMIT (k > 16384),
 * JET_EGRAPH (malformed CSR), JET_ENOMEM. Waits on `stream` a few times
 * (one look per four relaxation passes). */
int jet_bfs_start(jet_context *ctx, const jet_csr *g, int32_t k, int32_t *part, void *stream);

/* ---- measurement ------------------------------------------------------------
 * The floor of a pass that reads every CSR entry of g (neighbour id, edge
 * weight when given) and gathers the neighbour's part: times one kernel that
 * does only that, with the partition held as refinement holds it for k parts
 * (one byte per vertex when k <= 256, else 16 bits), reps times after one
 * warm-up, and writes the average milliseconds to *ms (host). `part`: device
 * int32[n] with every entry in [0, k). Returns JET_EINVAL (NULL pointers,
 * reps < 1, k < 1), JET_ELIMIT (k > 16384); the graph's ids are checked
 * first (JET_EGRAPH). Its algorithmic traffic is 4 nnz (8 nnz with edge
 * weights) + n (k <= 256) or 2 n bytes. */
int jet_gather_ceiling(jet_context *ctx, const jet_csr *g, const int32_t *part, int32_t k, int32_t reps, float *ms,
                       void *stream);

/* ---- serving loop ---------------------------------------------------------
 * A server partitions submitted jobs (each one jet_partition call's worth of
 * work) with continuous batching at level granularity. A worker thread owns
 * the context and a stream of its own and repeats one step:
 *   1. admit queued jobs in submission order while fewer than max_slots are
 *      active and the job's HBM footprint fits in what the budget has left;
 *      an admitted job is checked, coarsened (its hierarchy stays in device
 *      memory until the job ends) and gets its coarsest start (seeded random,
 *      or graph-growing with JET_F_BFS_START);
 *   2. refine the current level of every active job in one jet_refine_batch
 *      launch sequence;
 *   3. project every job one level finer; a job whose finest level was
 *      refined is done: its hierarchy is freed and its budget returned.
 * Jobs therefore join and leave the device-wide batch between steps, and a
 * job's result does not depend on what else is in the batch: it equals
 * jet_partition(graph, params) bit for bit.
 * Footprint of a job (bytes): 3 (8 (n+1) + 4 nnz (1 + [adjwgt]) + 4 n [vwgt])
 * + 48 n: its level graphs, its share of the batch's union copies and
 * per-vertex state, and two partition buffers.
 * The context belongs to the server until jet_server_destroy; the caller
 * must not use it meanwhile. Submit, poll and wait are thread-safe. */
typedef struct jet_server jet_server;

typedef struct {
    jet_csr graph;          /* device CSR, valid and unchanged until the job is done */
    jet_params params;      /* as for jet_partition (JET_F_PROFILE ignored) */
    int32_t *part_out;      /* device int32[n]; holds the partition once the job is done */
} jet_job;

typedef struct {
    int32_t status;         /* JET_OK, or the error that ended the job */
    int32_t levels;         /* hierarchy levels */
    int32_t iters;          /* refinement iterations over all levels */
    int32_t balanced;
    int64_t cut, max_part_weight;
    double t_submit_ms;     /* host steady clock, ms since the server was created */
    double t_admit_ms;
    double t_done_ms;
    int32_t steps;          /* batch steps the job took part in */
    int32_t reserved;
} jet_result;

typedef struct {
    int64_t submitted, completed, steps;
    int64_t step_jobs;      /* sum over steps of the number of jobs refined together */
    int32_t active, queued;
    int64_t hbm_in_use;     /* footprint of the active jobs (bytes) */
    double busy_ms;         /* host time the worker spent in steps */
} jet_server_info;

/* hbm_budget_bytes: total footprint of the jobs active at once (0 = no
 * limit); max_slots: jobs active at once (>= 1). The queue holds at most
 * 65536 jobs. */
int jet_server_create(jet_server **server, jet_context *ctx, size_t hbm_budget_bytes, int32_t max_slots);
/* Queues a job; *ticket identifies it. JET_EAGAIN: queue full; JET_ELIMIT:
 * the job's footprint exceeds the whole budget; JET_EINVAL / JET_ELIMIT for
 * parameters jet_partition would reject up front. */
int jet_server_submit(jet_server *server, const jet_job *job, uint64_t *ticket);
/* JET_OK and *result once the job is done (the ticket is then released),
 * JET_EAGAIN while it is not, JET_EINVAL for an unknown ticket. */
int jet_server_poll(jet_server *server, uint64_t ticket, jet_result *result);
/* As poll, but waits up to timeout_ms (< 0: no limit) for the job to end. */
int jet_server_wait(jet_server *server, uint64_t ticket, int32_t timeout_ms, jet_result *result);
int jet_server_info_get(jet_server *server, jet_server_info *info);
/* Finishes every submitted job, then stops the worker and frees the server
 * (results not yet polled are dropped). */
void jet_server_destroy(jet_server *server);

#ifdef __cplusplus
}
#endif
#endif /* JET_H */
