// Serving loop: continuous batching of multilevel partition jobs at level
// granularity (Algorithm 1 per job; every level's refinement, Algorithm 3,
// runs inside a batch shared by the active jobs of a lane).
//
// Jobs wait in one queue and are admitted in submission order while slots
// and the HBM budget allow (jet_sched.h). An admitted job goes to a lane: a
// worker thread with its own context, stream and memory pool. Lane 0 batches
// the small jobs; larger jobs go to the other lanes, so a large job's level
// never gates the small jobs' steps and large jobs overlap on the device.
// Each lane step starts its newly admitted jobs (checks, coarsening, the
// coarsest start; the hierarchy stays in device memory), refines the current
// level of every active job of the lane in one batched launch sequence, then
// projects each job one level finer or retires it. Because a batch refines
// each graph exactly as it would alone, a job's result is that of
// jet_partition on its own.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "jet_internal.h"
#include "jet_sched.h"

namespace jet {

constexpr size_t QUEUE_CAP = 65536;

struct SJob {
    uint64_t ticket = 0;
    jet_job spec;
    size_t footprint = 0;
    jet_hierarchy h;
    bool has_h = false;
    int32_t *buf = nullptr;  // two coarse partition buffers of n_1 ints each
    hipMemPool_t pool = nullptr;  // where buf came from (nullptr: hipMalloc)
    hipStream_t pool_stream = nullptr;
    int32_t *cur = nullptr;  // partition of the current level
    int level = 0;           // level refined by the next step
    jet_result res;
    jet_stats fin;           // stats of the finest level
};

static size_t job_footprint(const jet_csr &g)
{
    return sched::job_footprint(g.n, g.nnz, g.vwgt != nullptr, g.adjwgt != nullptr);
}

// One lane: a worker thread with its own context, stream and memory pool.
// Lane 0 batches (it takes every job of its inbox); the others run one job
// at a time from the server's shared queue of admitted large jobs.
struct Lane {
    int id = 0;
    bool batch = true;
    jet_context *ctx = nullptr;
    bool own_ctx = false;
    hipStream_t stream = nullptr;
    hipMemPool_t pool = nullptr;                 // stream-ordered job memory of this lane
    std::deque<std::unique_ptr<SJob>> inbox;     // batch lane: admitted, not yet started (server lock)
    std::condition_variable cv;
    std::thread th;
};

}  // namespace jet

struct jet_server {
    jet_context *ctx = nullptr;
    size_t budget = 0;
    int max_slots = 1;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_done;  // waiters: a job finished
    std::deque<std::unique_ptr<jet::SJob>> queue;
    std::unordered_map<uint64_t, jet_result> done;
    std::unordered_map<uint64_t, int> pending;  // submitted, not yet done
    std::vector<std::unique_ptr<jet::Lane>> lanes;
    std::deque<std::unique_ptr<jet::SJob>> large;  // admitted large jobs, for the single-job lanes
    size_t in_use = 0;      // footprint of the admitted jobs
    int active_total = 0;   // admitted jobs not yet retired
    uint64_t next_ticket = 1;
    bool stop = false;
    jet_server_info info;

    double now_ms() const
    {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace jet {

static void free_job(SJob *j)
{
    if (j->has_h) {
        hierarchy_release(&j->h);
        j->has_h = false;
    }
    if (j->buf) {
        if (j->pool) (void)hipFreeAsync(j->buf, j->pool_stream);
        else (void)hipFree(j->buf);
        j->buf = nullptr;
    }
}

// Checks, coarsens and seeds an admitted job; on return j->cur holds the
// coarsest level's partition and j->level is that level.
static int start_job(Lane *ln, SJob *j)
{
    jet_context *ctx = ln->ctx;
    hipStream_t s = ln->stream;
    const jet_csr &g = j->spec.graph;
    const jet_params &p = j->spec.params;
    int st = check_graph(ctx, &g, p.flags, s);
    if (st) return st;
    j->h.pool = ln->pool;
    j->h.pool_stream = s;
    j->pool = ln->pool;
    j->pool_stream = s;
    st = hierarchy_build(ctx, &g, &p, &j->h, s);
    j->has_h = true;
    if (st) return st;
    const int L = j->h.nlevels;
    const int l = L - 1;
    j->level = l;
    if (l == 0) {
        j->cur = j->spec.part_out;
    } else {
        const size_t n1 = (size_t)std::max(j->h.lv[1].n, 1);
        const hipError_t e = ln->pool ? hipMallocFromPoolAsync((void **)&j->buf, 2 * n1 * sizeof(int32_t), ln->pool, s)
                                      : hipMalloc((void **)&j->buf, 2 * n1 * sizeof(int32_t));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            j->buf = nullptr;
            return JET_ENOMEM;
        }
        // the coarsest level uses the half the next-finer level will not write to
        j->cur = (l % 2 == 1) ? j->buf : j->buf + n1;
    }
    st = coarsest_start(ctx, &j->h.lv[l], &p, j->cur, s);
    if (st) return st;
    j->res.levels = L;
    return JET_OK;
}

// Projects a job's partition one level finer (into part_out at level 0).
static int step_down(Lane *ln, SJob *j)
{
    const int l = j->level;
    const size_t n1 = (size_t)std::max(j->h.lv[1].n, 1);
    int32_t *dst = l - 1 == 0 ? j->spec.part_out : ((l - 1) % 2 == 1 ? j->buf : j->buf + n1);
    const int st = project_partition(ln->ctx, j->h.lv[l - 1].n, j->h.maps[l - 1], j->cur, dst, ln->stream);
    if (st) return st;
    j->cur = dst;
    j->level = l - 1;
    return JET_OK;
}

// Admits queued jobs in submission order while slots and the budget allow
// and hands each to its lane. Called with the server lock held.
static void admit_locked(jet_server *sv)
{
    const int nl = (int)sv->lanes.size();
    while (!sv->queue.empty()) {
        SJob *j = sv->queue.front().get();
        if (!sched::may_admit(j->footprint, sv->active_total, sv->max_slots, sv->in_use, sv->budget)) break;
        sv->in_use += j->footprint;
        sv->active_total++;
        j->res.t_admit_ms = sv->now_ms();
        if (sched::batch_lane_job(j->spec.graph.nnz, nl)) {
            sv->lanes[0]->inbox.push_back(std::move(sv->queue.front()));
            sv->lanes[0]->cv.notify_one();
        } else {
            sv->large.push_back(std::move(sv->queue.front()));
            for (int l = 1; l < nl; l++) sv->lanes[l]->cv.notify_one();
        }
        sv->queue.pop_front();
    }
    sv->info.queued = (int32_t)sv->queue.size();
    sv->info.active = sv->active_total;
    sv->info.hbm_in_use = (int64_t)sv->in_use;
    if (sv->stop && sv->queue.empty() && sv->large.empty())
        for (auto &l : sv->lanes) l->cv.notify_all();
}

static void lane_main(jet_server *sv, Lane *ln)
{
    (void)hipSetDevice(ln->ctx->device);
    std::vector<std::unique_ptr<SJob>> active;
    for (;;) {
        std::vector<std::unique_ptr<SJob>> admitted;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            // a stopping server still finishes every queued job: a lane leaves
            // only once the queue is empty (some lane has work while it is not)
            auto ready = [&] { return ln->batch ? !ln->inbox.empty() : (active.empty() && !sv->large.empty()); };
            auto leave = [&] {
                return sv->stop && sv->queue.empty() && sv->large.empty() && ln->inbox.empty() && active.empty();
            };
            ln->cv.wait(lk, [&] { return ready() || !active.empty() || leave(); });
            if (leave()) break;
            if (ln->batch) {
                while (!ln->inbox.empty()) {
                    admitted.push_back(std::move(ln->inbox.front()));
                    ln->inbox.pop_front();
                }
            } else if (active.empty() && !sv->large.empty()) {
                admitted.push_back(std::move(sv->large.front()));
                sv->large.pop_front();
            }
        }
        const double t_step = sv->now_ms();
        std::vector<std::unique_ptr<SJob>> finished;
        for (auto &j : admitted) {
            const int st = start_job(ln, j.get());
            if (st) {
                j->res.status = st;
                finished.push_back(std::move(j));
            } else {
                active.push_back(std::move(j));
            }
        }
        int m = (int)active.size();
        if (m > 0) {
            std::vector<jet_csr> graphs(m);
            std::vector<jet_params> params(m);
            std::vector<int32_t *> parts(m);
            std::vector<jet_stats> stats(m);
            for (int i = 0; i < m; i++) {
                SJob *j = active[i].get();
                graphs[i] = j->h.lv[j->level];
                params[i] = j->spec.params;
                params[i].level = j->level;
                params[i].flags &= ~(uint32_t)(JET_F_VALIDATE | JET_F_PROFILE);
                parts[i] = j->cur;
            }
            // one job: the single-graph refinement (its own fast paths, no
            // union copy); several: one batched launch sequence. Both give
            // each graph the result it would get alone.
            const int st = m == 1 ? refine_level(ln->ctx, &graphs[0], &params[0], parts[0], nullptr, &stats[0],
                                                 nullptr, 0, nullptr, nullptr, ln->stream)
                                  : refine_batch(ln->ctx, m, graphs.data(), params.data(), parts.data(),
                                                 stats.data(), nullptr, ln->stream);
            std::vector<std::unique_ptr<SJob>> still;
            for (int i = 0; i < m; i++) {
                std::unique_ptr<SJob> &j = active[i];
                j->res.steps++;
                int js = st;
                bool last = false;
                if (js == JET_OK) {
                    j->res.iters += stats[i].iters;
                    if (j->level == 0) {
                        j->fin = stats[i];  // the finest level was refined: the job is done
                        last = true;
                    } else {
                        js = step_down(ln, j.get());
                    }
                }
                if (js != JET_OK) j->res.status = js;
                if (js != JET_OK || last) finished.push_back(std::move(j));
                else still.push_back(std::move(j));
            }
            active.swap(still);
        }
        // projections of the step must be complete before a job is reported
        (void)hipStreamSynchronize(ln->stream);
        const double t_end = sv->now_ms();
        for (auto &j : finished) {
            if (j->res.status == JET_OK) {
                j->res.cut = j->fin.cut;
                j->res.max_part_weight = j->fin.max_part_weight;
                j->res.balanced = j->fin.balanced;
            }
            j->res.t_done_ms = t_end;
            free_job(j.get());
        }
        std::lock_guard<std::mutex> lk(sv->mu);
        if (m > 0) {
            sv->info.steps++;
            sv->info.step_jobs += m;
        }
        sv->info.busy_ms += t_end - t_step;
        for (auto &j : finished) {
            sv->in_use -= j->footprint;
            sv->active_total--;
            sv->done[j->ticket] = j->res;
            sv->pending.erase(j->ticket);
            sv->info.completed++;
        }
        if (!finished.empty()) {
            admit_locked(sv);  // budget and slots were returned
            sv->cv_done.notify_all();
        }
        sv->info.active = sv->active_total;
        sv->info.hbm_in_use = (int64_t)sv->in_use;
    }
}

}  // namespace jet

using namespace jet;

static void lane_release(Lane *ln)
{
    if (ln->stream) {
        (void)hipSetDevice(ln->ctx->device);
        (void)hipStreamSynchronize(ln->stream);
    }
    if (ln->pool) (void)hipMemPoolDestroy(ln->pool);
    if (ln->stream) (void)hipStreamDestroy(ln->stream);
    if (ln->own_ctx) jet_context_destroy(ln->ctx);
}

extern "C" int jet_server_create(jet_server **out, jet_context *ctx, size_t hbm_budget_bytes, int32_t max_slots)
{
    if (!out || !ctx || max_slots < 1) return JET_EINVAL;
    *out = nullptr;
    jet_server *sv = new (std::nothrow) jet_server();
    if (!sv) return JET_ENOMEM;
    sv->ctx = ctx;
    sv->budget = hbm_budget_bytes;
    sv->max_slots = max_slots;
    sv->t0 = std::chrono::steady_clock::now();
    memset(&sv->info, 0, sizeof(sv->info));
    int nl = sched::lane_count(max_slots);
    // JET_SERVER_LANES=n caps the lanes (tuning and measurement)
    if (const char *e = getenv("JET_SERVER_LANES")) {
        const int want = atoi(e);
        if (want >= 1 && want < nl) nl = want;
    }
    int st = JET_OK;
    for (int l = 0; l < nl && st == JET_OK; l++) {
        std::unique_ptr<Lane> ln(new (std::nothrow) Lane());
        if (!ln) {
            st = JET_ENOMEM;
            break;
        }
        ln->id = l;
        ln->batch = l == 0;
        // lane 0 runs on the caller's context, the others on their own
        if (l == 0) ln->ctx = ctx;
        else {
            st = jet_context_create(&ln->ctx, ctx->device);
            if (st) break;
            ln->own_ctx = true;
        }
        hipError_t e = hipSetDevice(ctx->device);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&ln->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            st = hip_status(ctx, e);
            lane_release(ln.get());
            break;
        }
        // job memory comes from a private stream-ordered pool that keeps what
        // it has (no device-wide wait per freed hierarchy); without one,
        // plain allocations are used
        hipMemPoolProps props;
        memset(&props, 0, sizeof(props));
        props.allocType = hipMemAllocationTypePinned;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = ctx->device;
        if (hipMemPoolCreate(&ln->pool, &props) == hipSuccess) {
            uint64_t keep = UINT64_MAX;
            (void)hipMemPoolSetAttribute(ln->pool, hipMemPoolAttrReleaseThreshold, &keep);
        } else {
            (void)hipGetLastError();
            ln->pool = nullptr;
        }
        sv->lanes.push_back(std::move(ln));
    }
    if (st == JET_OK) {
        try {
            for (auto &ln : sv->lanes) ln->th = std::thread(lane_main, sv, ln.get());
        } catch (...) {
            st = JET_ENOMEM;
        }
    }
    if (st != JET_OK) {
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->stop = true;
        }
        for (auto &ln : sv->lanes) {
            ln->cv.notify_all();
            if (ln->th.joinable()) ln->th.join();
            lane_release(ln.get());
        }
        delete sv;
        return st;
    }
    *out = sv;
    return JET_OK;
}

extern "C" int jet_server_submit(jet_server *sv, const jet_job *job, uint64_t *ticket)
{
    if (!sv || !job || !ticket) return JET_EINVAL;
    const jet_csr &g = job->graph;
    const jet_params &p = job->params;
    if (p.k < 1 || p.lambda_ppm < 0 || g.n < 0 || g.nnz < 0 || (g.n > 0 && (!job->part_out || !g.xadj)) ||
        (g.nnz > 0 && !g.adjncy) || (p.flags & JET_F_ASYNC))
        return JET_EINVAL;
    if (p.k > KMAX) return JET_ELIMIT;
    std::unique_ptr<SJob> j(new (std::nothrow) SJob());
    if (!j) return JET_ENOMEM;
    j->spec = *job;
    j->footprint = job_footprint(g);
    if (!sched::fits_alone(j->footprint, sv->budget)) return JET_ELIMIT;
    memset(&j->res, 0, sizeof(j->res));
    memset(&j->fin, 0, sizeof(j->fin));
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return JET_EINVAL;
    if (sv->queue.size() >= QUEUE_CAP) return JET_EAGAIN;
    j->ticket = sv->next_ticket++;
    j->res.t_submit_ms = sv->now_ms();
    *ticket = j->ticket;
    sv->pending[j->ticket] = 1;
    sv->queue.push_back(std::move(j));
    sv->info.submitted++;
    admit_locked(sv);
    return JET_OK;
}

static int take_result(jet_server *sv, uint64_t ticket, jet_result *result)
{
    auto it = sv->done.find(ticket);
    if (it != sv->done.end()) {
        if (result) *result = it->second;
        sv->done.erase(it);
        return JET_OK;
    }
    return sv->pending.count(ticket) ? JET_EAGAIN : JET_EINVAL;
}

extern "C" int jet_server_poll(jet_server *sv, uint64_t ticket, jet_result *result)
{
    if (!sv) return JET_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    return take_result(sv, ticket, result);
}

extern "C" int jet_server_wait(jet_server *sv, uint64_t ticket, int32_t timeout_ms, jet_result *result)
{
    if (!sv) return JET_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto ready = [&] { return sv->done.count(ticket) || !sv->pending.count(ticket); };
    if (timeout_ms < 0) sv->cv_done.wait(lk, ready);
    else sv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
    return take_result(sv, ticket, result);
}

extern "C" int jet_server_info_get(jet_server *sv, jet_server_info *info)
{
    if (!sv || !info) return JET_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    *info = sv->info;
    return JET_OK;
}

extern "C" void jet_server_destroy(jet_server *sv)
{
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        // queued jobs are admitted as lanes retire jobs; wake every lane
        for (auto &ln : sv->lanes) ln->cv.notify_all();
    }
    for (auto &ln : sv->lanes)
        if (ln->th.joinable()) ln->th.join();
    for (auto &ln : sv->lanes) lane_release(ln.get());
    delete sv;
}
