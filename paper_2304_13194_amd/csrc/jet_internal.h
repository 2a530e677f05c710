// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/jet.h"

namespace jet {

constexpr int NSLOT = 33;   // loss slots 0..32: losses are int32 (|loss| <= weighted degree < 2^31)
constexpr int KMAX = 16384; // part-count limit (dense LDS tables of int32)
constexpr int BLOCK = 256;  // threads per block of the row kernels
constexpr int TILE = 2048;  // vertices per tile of the ordered-selection kernels (one wave each)
// Per-block partial counters: slot 0 |X| (Jetlp) or eligible count (rebalancing),
// 1 |M|, 2 cut change, 3 moved weight, 4 digest change.
// Profiling counters of the gain pass: 5 CSR entries of unlocked rows, 6 unlocked
// rows, 7 visited vertices.
enum Stat { ST_X = 0, ST_M = 1, ST_DCUT = 2, ST_MW = 3, ST_DIG = 4, ST_E = 5, ST_R = 6, ST_V = 7, NSTAT = 8 };
constexpr int KIND_LOG = 1 << 16;  // iterations whose kind is logged
constexpr int NSHARD = 64;  // shards per counter row

enum Kind { KIND_DONE = 0, KIND_LP = 1, KIND_RW = 2, KIND_RS = 3 };
// Degree classes: 0 isolated, 1 small (<= 32), 2 medium (<= 1024), 3 large.
enum Cls { CLS_Z = 0, CLS_S = 1, CLS_M = 2, CLS_L = 3, NCLS = 4 };
constexpr int S_MAXDEG = 32;
constexpr int M_MAXDEG = 1024;

// Device-resident loop state of one refinement call.
struct Ctl {
    // configuration (written by the host before the first iteration)
    int32_t n, k, stall_limit, bmax;
    int32_t max_iters, c_num, c_den, phi_num;
    int32_t phi_den, level, trace_cap, nB;
    int64_t W, o, sigma;
    uint64_t seed;
    // loop state
    int32_t kind, t, stall, wcount;
    int32_t lp_id, done, balanced, bal_best;
    int32_t copy_best, nA, nsplit, n_lp;
    int32_t n_rw, n_rs, err, pad0;
    int64_t cut, cut_best, maxw, maxw_best;
    uint64_t digest;
    // per-iteration results (reduced from per-block partials)
    int32_t nX, nM;
    int64_t dcut, moved_w;
    uint64_t ddigest;
    int64_t total_cap;
    // set-up accumulators
    int64_t wsum, ewsum;
    int64_t prof_e, prof_r, prof_v;  // gain-pass counters summed over Jetlp iterations
    int32_t bincnt[NCLS];
    int32_t bad_graph, bad_part;
};

// Everything a kernel needs, passed by value.
struct KArgs {
    int32_t n, k;
    const int64_t *xadj;
    const int32_t *adj;
    const int32_t *vw;
    const int32_t *ew;
    int32_t *P;      // P_iter
    int32_t *best;   // P_best (the caller's array)
    int2 *rec;       // per-vertex Jetlp record: x = (P_s << 16) | (in X ? P_d + 1 : 0), y = F
    int32_t *dest;   // move destination or -1 (kept -1 outside moves)
    int32_t *lock;   // Jetlp id of the last move of each vertex
    uint8_t *slot;   // rebalancing loss slot, 255 = not a candidate
    int32_t *rbd;    // Jetrw destination of each candidate
    uint8_t *rsev;   // Jetrs: evicted flag
    const int32_t *bins;   // vertex ids grouped by degree class
    int32_t binoff[NCLS + 1];
    int64_t *bstat;  // iteration counters [NSTAT][NSHARD], summed by the controller
    int32_t grid_tab, grid_rbtab, grid_plain;
    Ctl *ctl;
    int64_t *w, *wbest, *resid, *capstart, *hist;
    int64_t *xbase;   // per split index: cut-off-slot weight before its crossing tile
    int32_t *Blist, *sstar, *splitidx;
    int32_t *splitpart, *xtile, *vthr;  // split index -> part, crossing tile; per part threshold id
    uint8_t *isA, *isB;
    int32_t *tsum;
    int64_t *esum;
    int32_t ntile;
    jet_trace_rec *trace;
    int8_t *kinds;   // kind of iteration t (t < KIND_LOG)
    // block counts per role of the row kernels
    int32_t gS, gM, gL, gZ;
    // which role (1 S, 2 M, 3 L) serves each class in the LDS-table kernels
    int32_t tmap[NCLS];
    int32_t ngroups_tab_S; // groups per block of the S role in table kernels
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

struct jet_context {
    int device = 0;
    int num_cu = 256;
    int last_hip = 0;
    std::vector<jet::Buffer> bufs;
    void *pinned = nullptr;  // host staging for small read-backs
    size_t pinned_bytes = 0;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<hipEvent_t> prof_ev;  // pairs around gain passes (JET_F_PROFILE)
};

namespace jet {

enum WsSlot {
    WS_P, WS_REC, WS_DEST, WS_LOCK, WS_SLOT, WS_RBD, WS_RSEV, WS_BIN, WS_BSTAT, WS_FILL,
    WS_CTL, WS_PART64, WS_PART32, WS_PART8, WS_HIST, WS_TSUM, WS_ESUM, WS_TRACE,
    WS_DBG_LOCK, WS_H0, WS_H1, WS_C0, WS_C1, WS_C2, WS_C3, WS_C4, WS_C5, WS_C6, WS_C7, WS_C8,
    WS_C9, WS_C10, WS_C11, WS_KINDS, WS_C12, WS_COUNT = 64
};

// Grow-only workspace slot; returns nullptr on allocation failure.
void *ws_get(jet_context *ctx, int slot, size_t bytes);

// Refinement of one level; `part` holds P_0 on entry and P_best on exit.
// `trace_dev`/`trace_cap` optional. stats filled (host). Stream already set.
int refine_level(jet_context *ctx, const jet_csr *g, const jet_params *prm, int32_t *part,
                 int64_t *part_weights_out, jet_stats *stats, jet_trace_rec *trace_host,
                 int32_t trace_cap, int32_t *trace_count, int32_t *trace_total, hipStream_t s);

int hip_status(jet_context *ctx, hipError_t e);

}  // namespace jet
