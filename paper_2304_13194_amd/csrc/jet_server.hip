// Serving loop: continuous batching of multilevel partition jobs at level
// granularity (Algorithm 1 per job; every level's refinement, Algorithm 3,
// runs inside one device-wide batch shared by all active jobs).
//
// A worker thread owns the context and its own stream. Each step admits
// queued jobs (slots and HBM footprint permitting; an admitted job is
// checked, coarsened, and given its coarsest start (seeded random or graph-growing), and its
// hierarchy stays in device memory), refines the current level of every
// active job in one batched launch sequence, then projects each job one
// level finer or retires it. Because a batch refines each graph exactly as
// it would alone, a job's result is that of jet_partition on its own.
#include <hip/hip_runtime.h>
#include <stdint.h>
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
    const size_t n = (size_t)std::max(g.n, 0), m = (size_t)std::max<int64_t>(g.nnz, 0);
    const size_t csr = 8 * (n + 1) + 4 * m * (g.adjwgt ? 2 : 1) + (g.vwgt ? 4 * n : 0);
    return 3 * csr + 48 * n;
}

}  // namespace jet

struct jet_server {
    jet_context *ctx = nullptr;
    hipStream_t stream = nullptr;
    hipMemPool_t pool = nullptr;  // stream-ordered job memory (hierarchies, partition buffers)
    size_t budget = 0;
    int max_slots = 1;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work;  // worker: new jobs or stop
    std::condition_variable cv_done;  // waiters: a job finished
    std::deque<std::unique_ptr<jet::SJob>> queue;
    std::unordered_map<uint64_t, jet_result> done;
    std::unordered_map<uint64_t, int> pending;  // submitted, not yet done
    uint64_t next_ticket = 1;
    bool stop = false;
    jet_server_info info;
    std::thread worker;

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
static int start_job(jet_server *sv, SJob *j)
{
    jet_context *ctx = sv->ctx;
    hipStream_t s = sv->stream;
    const jet_csr &g = j->spec.graph;
    const jet_params &p = j->spec.params;
    int st = check_graph(ctx, &g, p.flags, s);
    if (st) return st;
    j->h.pool = sv->pool;
    j->h.pool_stream = s;
    j->pool = sv->pool;
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
        const hipError_t e = sv->pool ? hipMallocFromPoolAsync((void **)&j->buf, 2 * n1 * sizeof(int32_t), sv->pool, s)
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
static int step_down(jet_server *sv, SJob *j)
{
    const int l = j->level;
    const size_t n1 = (size_t)std::max(j->h.lv[1].n, 1);
    int32_t *dst = l - 1 == 0 ? j->spec.part_out : ((l - 1) % 2 == 1 ? j->buf : j->buf + n1);
    const int st = project_partition(sv->ctx, j->h.lv[l - 1].n, j->h.maps[l - 1], j->cur, dst, sv->stream);
    if (st) return st;
    j->cur = dst;
    j->level = l - 1;
    return JET_OK;
}

static void worker_main(jet_server *sv)
{
    (void)hipSetDevice(sv->ctx->device);
    std::vector<std::unique_ptr<SJob>> active;
    size_t in_use = 0;
    for (;;) {
        std::vector<std::unique_ptr<SJob>> admitted;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_work.wait(lk, [&] { return sv->stop || !sv->queue.empty() || !active.empty(); });
            if (sv->stop && sv->queue.empty() && active.empty()) break;
            while (!sv->queue.empty() && (int)(active.size() + admitted.size()) < sv->max_slots) {
                const size_t f = sv->queue.front()->footprint;
                if (sv->budget && in_use + f > sv->budget) break;
                in_use += f;
                admitted.push_back(std::move(sv->queue.front()));
                sv->queue.pop_front();
            }
            sv->info.queued = (int32_t)sv->queue.size();
        }
        const double t_step = sv->now_ms();
        std::vector<std::unique_ptr<SJob>> finished;
        for (auto &j : admitted) {
            j->res.t_admit_ms = sv->now_ms();
            const int st = start_job(sv, j.get());
            if (st) {
                j->res.status = st;
                finished.push_back(std::move(j));
            } else {
                active.push_back(std::move(j));
            }
        }
        if (!active.empty()) {
            const int m = (int)active.size();
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
            const int st = refine_batch(sv->ctx, m, graphs.data(), params.data(), parts.data(), stats.data(), nullptr,
                                        sv->stream);
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
                        js = step_down(sv, j.get());
                    }
                }
                if (js != JET_OK) j->res.status = js;
                if (js != JET_OK || last) finished.push_back(std::move(j));
                else still.push_back(std::move(j));
            }
            active.swap(still);
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->info.steps++;
            sv->info.step_jobs += m;
        }
        // projections of the step must be complete before a job is reported
        (void)hipStreamSynchronize(sv->stream);
        const double t_end = sv->now_ms();
        for (auto &j : finished) {
            if (j->res.status == JET_OK) {
                j->res.cut = j->fin.cut;
                j->res.max_part_weight = j->fin.max_part_weight;
                j->res.balanced = j->fin.balanced;
            }
            j->res.t_done_ms = t_end;
            free_job(j.get());
            in_use -= j->footprint;
        }
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->info.busy_ms += t_end - t_step;
        sv->info.active = (int32_t)active.size();
        sv->info.hbm_in_use = (int64_t)in_use;
        for (auto &j : finished) {
            sv->done[j->ticket] = j->res;
            sv->pending.erase(j->ticket);
            sv->info.completed++;
        }
        if (!finished.empty()) sv->cv_done.notify_all();
    }
}

}  // namespace jet

using namespace jet;

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
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        const int st = hip_status(ctx, e);
        delete sv;
        return st;
    }
    // job memory comes from a private stream-ordered pool that keeps what it
    // has (no device-wide wait per freed hierarchy); without one, plain
    // allocations are used
    {
        hipMemPoolProps props;
        memset(&props, 0, sizeof(props));
        props.allocType = hipMemAllocationTypePinned;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = ctx->device;
        if (hipMemPoolCreate(&sv->pool, &props) == hipSuccess) {
            uint64_t keep = UINT64_MAX;
            (void)hipMemPoolSetAttribute(sv->pool, hipMemPoolAttrReleaseThreshold, &keep);
        } else {
            (void)hipGetLastError();
            sv->pool = nullptr;
        }
    }
    try {
        sv->worker = std::thread(worker_main, sv);
    } catch (...) {
        if (sv->pool) (void)hipMemPoolDestroy(sv->pool);
        (void)hipStreamDestroy(sv->stream);
        delete sv;
        return JET_ENOMEM;
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
        (g.nnz > 0 && !g.adjncy))
        return JET_EINVAL;
    if (p.k > KMAX) return JET_ELIMIT;
    std::unique_ptr<SJob> j(new (std::nothrow) SJob());
    if (!j) return JET_ENOMEM;
    j->spec = *job;
    j->footprint = job_footprint(g);
    if (sv->budget && j->footprint > sv->budget) return JET_ELIMIT;
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
    sv->info.queued = (int32_t)sv->queue.size();
    sv->cv_work.notify_one();
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
        sv->cv_work.notify_all();
    }
    if (sv->worker.joinable()) sv->worker.join();
    (void)hipSetDevice(sv->ctx->device);
    (void)hipStreamSynchronize(sv->stream);
    if (sv->pool) (void)hipMemPoolDestroy(sv->pool);
    (void)hipStreamDestroy(sv->stream);
    delete sv;
}
