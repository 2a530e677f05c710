// Scheduling decisions of the serving loop, as pure functions: no HIP, no
// clock, no threads, so that a host-only build can drive them with a fake
// budget and a fake clock. jet_server.hip calls exactly these.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace jet {
namespace sched {

// HBM footprint of a job (bytes): its level graphs (the finest one plus
// coarse ones of at most the same size, three CSR copies in all), its share
// of the batch's union copies and per-vertex state, two partition buffers.
inline size_t job_footprint(int64_t n, int64_t nnz, bool has_vwgt, bool has_adjwgt)
{
    const size_t nn = (size_t)(n > 0 ? n : 0), m = (size_t)(nnz > 0 ? nnz : 0);
    const size_t csr = 8 * (nn + 1) + 4 * m * (has_adjwgt ? 2 : 1) + (has_vwgt ? 4 * nn : 0);
    return 3 * csr + 48 * nn;
}

// A job whose footprint alone exceeds a nonzero budget can never run.
inline bool fits_alone(size_t footprint, size_t budget) { return budget == 0 || footprint <= budget; }

// The job at the head of the queue is admitted when a slot is free and its
// footprint fits in what the budget has left (budget 0: no limit). Jobs are
// admitted strictly in submission order: a job that does not fit holds back
// every later one, so no large job waits forever behind smaller ones.
inline bool may_admit(size_t footprint, int active, int max_slots, size_t in_use, size_t budget)
{
    return active < max_slots && (budget == 0 || in_use + footprint <= budget);
}

// Lanes: lane 0 batches the small jobs (at most SMALL_NNZ CSR entries),
// level by level: their levels are cheap and their launches are what
// batching amortises. Every larger job runs alone on one of the other
// lanes, which take admitted large jobs one at a time, in admission order,
// from a queue they share: independent jobs on their own streams overlap on
// the device, and a large job neither gates a batch step (a step lasts as
// long as its slowest level) nor waits behind another lane's long job. With
// one lane, that lane batches everything.
constexpr int64_t SMALL_NNZ = (int64_t)1 << 18;

inline bool batch_lane_job(int64_t nnz, int nlanes) { return nlanes <= 1 || nnz <= SMALL_NNZ; }

// Lanes of a server with `max_slots` slots: the batch lane plus up to four
// single-job lanes (independent partitions stop gaining beyond about four
// concurrent streams on one MI355X).
constexpr int MAX_LANES = 5;
inline int lane_count(int max_slots) { return max_slots < 1 ? 1 : (max_slots > MAX_LANES ? MAX_LANES : max_slots); }

}  // namespace sched
}  // namespace jet
