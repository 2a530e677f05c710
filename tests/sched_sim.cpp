// Host-only event simulation of the serving loop's scheduling decisions
// (admission by slots and HBM budget in submission order; small jobs to the
// batch lane, larger ones to single-job lanes that take them one at a time,
// in admission order, from a shared queue), with a fake clock: job i arrives
// at arrival[i] ms and needs service[i] ms once started; it holds its slot
// and footprint from admission to completion. The decisions are jet_sched.h's,
// the functions jet_server.hip calls; only the clock and the service times are
// simulated. Built by the CPU tests with g++.
#include <stdint.h>

#include <deque>
#include <vector>

#include "jet_sched.h"

extern "C" int sched_simulate(int njobs, const double *arrival, const double *service, const int64_t *nnz,
                              const int64_t *footprint, int max_slots, uint64_t budget, double *admit,
                              double *start, double *done, int32_t *lane, int64_t *max_in_use, int32_t *max_active)
{
    using namespace jet::sched;
    const int nl = lane_count(max_slots);
    std::deque<int> queue, large;         // submitted; admitted large jobs waiting for a lane
    std::vector<int> busy(nl, -1);        // job running on each single-job lane
    std::vector<char> running(njobs, 0);
    int next = 0, active = 0, finished = 0;
    uint64_t in_use = 0;
    *max_in_use = 0;
    *max_active = 0;
    for (int i = 0; i < njobs; i++) {
        admit[i] = start[i] = done[i] = -1.0;
        lane[i] = -1;
        if (!fits_alone((size_t)footprint[i], (size_t)budget)) return -1 - i;  // rejected at submission
    }
    double now = 0.0;
    auto begin = [&](int j, int l) {
        lane[j] = l;
        start[j] = now;
        running[j] = 1;
        if (l > 0) busy[l] = j;
    };
    while (finished < njobs) {
        double t_arr = next < njobs ? arrival[next] : 1e300, t_done = 1e300;
        int who = -1;
        for (int i = 0; i < njobs; i++)
            if (running[i] && start[i] + service[i] < t_done) {
                t_done = start[i] + service[i];
                who = i;
            }
        if (t_arr <= t_done) {
            now = t_arr;
            queue.push_back(next++);
        } else {
            now = t_done;
            running[who] = 0;
            done[who] = now;
            active--;
            in_use -= (uint64_t)footprint[who];
            if (lane[who] > 0) busy[lane[who]] = -1;
            finished++;
        }
        // admission, as the server does after a submission or a retirement
        while (!queue.empty()) {
            const int j = queue.front();
            if (!may_admit((size_t)footprint[j], active, max_slots, (size_t)in_use, (size_t)budget)) break;
            in_use += (uint64_t)footprint[j];
            active++;
            admit[j] = now;
            queue.pop_front();
            if (batch_lane_job(nnz[j], nl)) begin(j, 0);
            else large.push_back(j);
            if ((int64_t)in_use > *max_in_use) *max_in_use = (int64_t)in_use;
            if (active > *max_active) *max_active = active;
        }
        // idle single-job lanes take the oldest admitted large job
        for (int l = 1; l < nl && !large.empty(); l++)
            if (busy[l] < 0) {
                begin(large.front(), l);
                large.pop_front();
            }
    }
    return nl;
}
