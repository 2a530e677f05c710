// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>
#include <vector>

#include "../../include/jet.h"

namespace jet {

constexpr int NSLOT = 33;    // loss slots 0..32: losses are int32 (|loss| <= weighted degree < 2^31)
constexpr int KMAX = 16384;  // part-count limit per graph (dense LDS tables of int32)
constexpr int BLOCK = 256;   // threads per block of the row kernels
constexpr int TILE = 2048;   // vertices per tile of the ordered-selection kernels
constexpr int PER = TILE / BLOCK;
// Iteration counters: 0 |X| (Jetlp) or eligible count (rebalancing), 1 |M|,
// 2 cut change, 3 moved weight, 4 digest change; profiling of the gain pass:
// 5 CSR entries of unlocked rows, 6 unlocked rows, 7 visited vertices.
enum Stat { ST_X = 0, ST_M = 1, ST_DCUT = 2, ST_MW = 3, ST_DIG = 4, ST_E = 5, ST_R = 6, ST_V = 7, NSTAT = 8 };
constexpr int NSHARD = 64;         // shards per counter row and graph
constexpr int KIND_LOG = 1 << 16;  // iterations whose kind is logged (graph 0)

enum Kind { KIND_DONE = 0, KIND_LP = 1, KIND_RW = 2, KIND_RS = 3 };
// Degree classes: 0 isolated, 1 small (<= 32), 2 small wide (<= 64), 3 medium
// (<= 1024), 4 large.
enum Cls { CLS_Z = 0, CLS_S = 1, CLS_S2 = 2, CLS_M = 3, CLS_L = 4, NCLS = 5 };
constexpr int S_MAXDEG = 32;
constexpr int S2_MAXDEG = 64;
constexpr int M_MAXDEG = 1024;

// Launch-wide counts: CNT_DONE graphs finished; then two rows (selected by
// the parity of the iteration's launch index) of [graphs whose previous
// iteration improved the best and that go on, graphs in Jetlp, Jetrw, Jetrs].
enum Cnt { CNT_DONE = 0, CNT_ROW = 2, CNT_N = 10, CNT_TFAIL = 11 };

// Device-resident state of one graph's refinement (one per graph of a batch).
struct Ctl {
    // configuration
    int32_t n, k, stall_limit, bmax;
    int32_t max_iters, c_num, c_den, phi_num;
    int32_t phi_den, level, trace_cap, nB;
    int32_t voff, poff, t0, ntiles;      // first vertex, first global part, first tile, tiles
    int32_t trace_off, flags, lambda_ppm, deadzone_div;
    int64_t W, o, sigma;
    int64_t rowbase;                     // first tile-sum entry of the graph
    uint64_t seed;
    // loop state
    int32_t kind, t, stall, wcount;
    int32_t lp_id, done, balanced, bal_best;
    int32_t copy_best, nA, n_lp, n_rw;
    int32_t n_rs, bad_part, nX, nM;
    int64_t cut, cut_best, maxw, maxw_best;
    uint64_t digest;
    // per-iteration results
    int64_t dcut, moved_w;
    uint64_t ddigest;
    int64_t total_cap;
    // set-up accumulators and profiling
    int64_t wsum, ewsum;
    int64_t prof_e, prof_r, prof_v;
};

// Everything a kernel needs, passed by value.
struct KArgs {
    int32_t n, k;          // union vertices; largest k of the batch (LDS table size)
    int32_t ngraph, ktot;  // graphs; total parts (global part id = poff + local part)
    const int64_t *xadj;
    const int32_t *adj;
    const int32_t *vw;
    const int32_t *ew;
    const int32_t *vg;     // graph of each vertex (NULL: one graph)
    const int32_t *pg;     // graph of each global part (NULL: one graph)
    const int32_t *tg;     // graph of each tile (NULL: one graph)
    uint16_t *P;           // P_iter (local part ids; k <= KMAX fits 16 bits, halving the gathered bytes)
    uint8_t *P8;           // P_iter again as bytes when every part id fits one (k <= 256; else NULL):
                           // the neighbour gathers of the row passes read it (half the footprint)
    void *mq;              // per vertex (P_iter, P_next) packed: bytes in a uint16 when k <= 256, else
                           // halves of a uint32; P_next = the selected destination, else P_iter.
                           // The cut-delta pass reads a neighbour's old and new part in one gather.
    uint32_t *rq;          // when P8: per vertex (P_s, in X ? P_d : P_s, F saturated to int16) in 4 bytes,
                           // the afterburner's neighbour gather (Fx only where saturation hides the
                           // order); it replaces rec, which is then neither written nor read.
                           // NULL: the afterburner gathers rec
    int32_t *Fx;           // with rq: the full F of the vertices of X (other entries stale)
    int32_t *best;         // P_best
    int2 *rec;             // Jetlp record: x = (P_s << 16) | (in X ? P_d + 1 : 0), y = F
    int32_t *dest;         // move destination or -1 (kept -1 outside moves)
    int32_t *lock;         // Jetlp id of the last move of each vertex
    uint8_t *slot;         // rebalancing loss slot, 255 = not a candidate
    int32_t *rbd;          // Jetrw destination of each candidate
    uint8_t *rsev;         // Jetrs: evicted flag
    const int32_t *bins;   // vertex ids grouped by degree class, ascending within a class
    int32_t binoff[NCLS + 1];
    int64_t *bstat;        // iteration counters [graph][NSTAT][NSHARD]
    Ctl *ctl;              // [ngraph]
    int32_t *cnt;          // [CNT_N] launch-wide counts
    int32_t it;            // launch index of the current iteration (its parity picks the count row)
    // per global part
    int64_t *w, *wbest, *resid, *hist;
    int64_t *capstart;     // Jetrs capacity starts: graph g's nB + 1 entries at poff + g
    int32_t *Blist, *sstar, *vthr;
    uint8_t *isA, *isB;
    int32_t *tsum;         // per graph: [k][ntiles] cut-off-slot weight per (part, tile)
    int64_t *esum;         // per tile: Jetrs evicted weight
    int32_t ntile;         // tiles (each inside one graph)
    jet_trace_rec *trace;
    int8_t *kinds;         // kind of iteration t of graph 0 (t < KIND_LOG)
    // block counts per role of the row kernels
    int32_t gS, gM, gL, gZ;
    int32_t gS2;           // blocks of the wide small-row kernels (class S2 in the small-row role)
    int32_t sident;        // one graph whose vertices all sit in the small class: its list is 0..n-1
    int32_t tmap[NCLS];    // which role (1 S, 2 M, 3 L) serves each class in the LDS-table kernels
    // long rows of the L class cut into chunks (see LCHUNK); nlch = 0: L rows use the block role
    const int2 *lch;       // (index in the L list, chunk index) per chunk
    const int32_t *lcoff;  // [L list + 1] first chunk of each long row
    int32_t nlch;
    int32_t lstride;       // row length of gconn (largest k)
    int32_t *gconn;        // [chunk][lstride] part counts of each chunk of a row of several chunks
    int32_t *ldone;        // [L list] chunks of the vertex completed in this pass
    int32_t *gf2;          // [L list] afterburner sum over a vertex's chunks
    // persistent connectivity table (one graph; toff NULL when off)
    const int64_t *toff;   // [n+1] first slot of each vertex's row; row v has min(k, deg v) slots
    unsigned long long *tab;  // slots: (count << 32) | part, or TAB_EMPTY
    int32_t *tsize;        // [n] slots of row v in use (its hash modulus)
    int32_t *tfail;        // [n] 1 while row v waits for its rebuild
    int32_t *tlist;        // rows to rebuild after this iteration's moves (count at cnt[CNT_TFAIL])
    // batch work queue: counters [2][NQ] (bank = launch parity); wtile visits
    // of a wave per tile (0: static walks)
    int32_t *wq;
    int32_t wtile;
    // optional step outputs
    int64_t *dbg_F, *dbg_cs, *dbg_F2, *dbg_loss;
    int32_t *dbg_pd;
    int32_t *dbg_slot;
};

struct Buffer {
    void *ptr = nullptr;
    size_t bytes = 0;
};

}  // namespace jet

namespace jet {
// Grow-only device arena: bump allocation from a list of chunks; reset()
// keeps the memory (merging the chunks into one when a call needed several),
// so repeated partitions of graphs of one size allocate nothing.
struct Arena {
    std::vector<Buffer> chunks;
    size_t cur = 0, used = 0;
    void *alloc(size_t bytes);
    void reset();
    void release();
};
}  // namespace jet

struct jet_hierarchy {
    int device = 0;
    int nlevels = 0;
    std::vector<jet_csr> lv;        // level views (level 0 = caller's graph)
    std::vector<int32_t *> maps;    // maps[l]: level l -> level l+1 (owned)
    std::vector<void *> owned;      // device buffers owned by the hierarchy (no arena)
    jet::Arena *arena = nullptr;    // when set, levels live in this arena instead
    hipMemPool_t pool = nullptr;    // else, when set: stream-ordered allocations from this pool
    hipStream_t pool_stream = nullptr;
    float ms_coarsen = 0.f;
};

struct jet_context {
    int device = 0;
    int num_cu = 256;
    int last_hip = 0;
    std::vector<jet::Buffer> bufs;
    void *pinned = nullptr;  // host staging for read-backs and controller uploads
    size_t pinned_bytes = 0;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<hipEvent_t> prof_ev;  // pairs around gain passes (JET_F_PROFILE)
    hipStream_t cap = nullptr;        // side stream on which iteration sequences are captured
    hipStream_t aux = nullptr;        // second stream of the contraction (hub rows beside the other rows)
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;  // fork to and join from aux
    bool graphs = true;               // replay captured iteration pairs (JET_NO_GRAPH=1 turns it off)
    hipEvent_t wait_ev = nullptr;     // polled by stream_wait
    jet::Arena part_arena;            // coarse levels of jet_partition calls
    bool poll_wait = true;            // poll instead of sleeping in the runtime (JET_BLOCKING_WAIT=1 turns it off)
    bool part8 = true;                // byte copy of P_iter for the gathers when k <= 256 (JET_NO_PART8=1 turns it off)
    // jet_refine_noalloc: device address of this device's static scratch
    // array (looked up once per device at context creation); while
    // scratch_on, ws_get carves its slots from it instead of allocating
    char *scratch = nullptr;
    size_t scratch_off = 0;
    bool scratch_on = false;
    // batch autotuner: chosen walk (tile | group-of-8 << 16) per batch shape
    std::vector<std::pair<uint64_t, int>> tune_cache;
};

namespace jet {

enum WsSlot {
    WS_P, WS_REC, WS_DEST, WS_LOCK, WS_SLOT, WS_RBD, WS_RSEV, WS_BIN, WS_BSTAT, WS_CNT,
    WS_CTL, WS_PART64, WS_PART32, WS_PART8, WS_HIST, WS_TSUM, WS_ESUM, WS_TRACE,
    WS_DBG_LOCK, WS_H0, WS_H1, WS_C0, WS_C1, WS_C2, WS_C3, WS_C4, WS_C5, WS_C6, WS_C7, WS_C8,
    WS_C9, WS_C10, WS_C11, WS_KINDS, WS_C12, WS_BLKCNT, WS_TG,
    WS_U_XADJ, WS_U_ADJ, WS_U_VW, WS_U_EW, WS_U_VG, WS_U_P0, WS_U_BEST, WS_U_DESC,
    WS_LCNT, WS_LCH, WS_GCONN, WS_LDONE, WS_TH_KEY, WS_TH_VAL, WS_TH_RUN, WS_TH_TMP, WS_WDEG,
    WS_TOFF, WS_TAB, WS_TSIZE, WS_TFAIL, WS_TLIST, WS_TBLK, WS_WQ, WS_TUNE_CTL, WS_TUNE_CNT, WS_TUNE_REC,
    WS_TUNE_STAT, WS_P8, WS_MQ, WS_RQ, WS_RMARK, WS_C13, WS_FX,
    WS_COUNT = 80
};
static_assert(WS_FX < WS_COUNT, "workspace slots");

// Grow-only workspace slot; returns nullptr on allocation failure.
void *ws_get(jet_context *ctx, int slot, size_t bytes);
// Grow-only pinned host staging; returns nullptr on allocation failure.
void *pinned_get(jet_context *ctx, size_t bytes);
// Waits for everything queued on s (polling an event, see jet_context).
hipError_t stream_wait(jet_context *ctx, hipStream_t s);

// Refinement of one level; `part` holds P_0 on entry and P_best on exit.
// cut0 >= 0: P_0 is the projection of a coarser level's result whose cut was
// cut0 (projection keeps the cut), and the graph is one the library built or
// checked, so the set-up skips its edge pass (cut, total edge weight and
// entry checks).
int refine_level(jet_context *ctx, const jet_csr *g, const jet_params *prm, int32_t *part,
                 int64_t *part_weights_out, jet_stats *stats, jet_trace_rec *trace_host,
                 int32_t trace_cap, int32_t *trace_count, int32_t *trace_total, hipStream_t s,
                 int64_t cut0 = -1);

// Refinement of `count` independent graphs in one launch sequence; parts[i]
// holds graph i's P_0 on entry and its P_best on exit.
int refine_batch(jet_context *ctx, int count, const jet_csr *graphs, const jet_params *params,
                 int32_t *const *parts, jet_stats *stats, jet_trace *traces, hipStream_t s);

int hip_status(jet_context *ctx, hipError_t e);
// Row marks of a CSR, for the passes that take runs of entries: mark[i] = the
// row holding entry i * MARK (the largest v with xadj[v] <= i * MARK), for
// i < nmark = nnz / MARK + 1, so that a run's row search starts within a few
// rows. Launched on s into workspace slot WS_RMARK.
constexpr int MARK = 4096;
int row_marks(jet_context *ctx, const int64_t *xadj, int n, int64_t nnz, int32_t **mark, int64_t *nmark,
              hipStream_t s);
int validate_full_csr(jet_context *ctx, const jet_csr *g, hipStream_t s);
// Cheap O(n + m) input checks (and the full check under JET_F_VALIDATE).
int check_graph(jet_context *ctx, const jet_csr *g, uint32_t flags, hipStream_t s);

// Multilevel scaffold: the hierarchy of g (levels owned by h until
// hierarchy_release), the seeded coarsest partition P[v] =
// floor(stream(mix64(seed ^ 1), v) k / 2^64), and projection to a finer level.
int hierarchy_build(jet_context *ctx, const jet_csr *g, const jet_params *prm, jet_hierarchy *h, hipStream_t s);
void hierarchy_release(jet_hierarchy *h);
int random_partition(jet_context *ctx, int n, int k, uint64_t seed, int32_t *part, hipStream_t s);
int bfs_start(jet_context *ctx, const jet_csr *g, int k, int32_t *part, hipStream_t s);
int coarsest_start(jet_context *ctx, const jet_csr *g, const jet_params *p, int32_t *part, hipStream_t s);
int project_partition(jet_context *ctx, int n, const int32_t *map, const int32_t *coarse, int32_t *fine, hipStream_t s);

}  // namespace jet
