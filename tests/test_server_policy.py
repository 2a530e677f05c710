"""CPU checks of the serving loop's scheduling decisions (jet_sched.h, the
functions jet_server.hip calls), driven by a host-only event simulation with
a fake clock (tests/sched_sim.cpp): admission never exceeds the HBM budget
or the slots, admits in submission order, holds jobs back while the budget
binds and admits every job eventually; small jobs batch in lane 0, larger
ones run one at a time per single-job lane, started in admission order; a
job larger than the whole budget is refused at submission."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

from paper_2304_13194_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "sched_sim.cpp")
INC = os.path.join(ROOT, "paper_2304_13194_amd", "csrc")
OUT = os.path.join(ROOT, "tests", "_build", "libschedsim.so")
SMALL_NNZ = 1 << 18


@pytest.fixture(scope="module")
def sim():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", INC, "-o", OUT, SRC])
    lib = C.CDLL(OUT)
    lib.sched_simulate.restype = C.c_int

    def run(arrival, service, nnz, fp, slots, budget):
        n = len(arrival)
        a = np.ascontiguousarray(arrival, np.float64)
        s = np.ascontiguousarray(service, np.float64)
        z = np.ascontiguousarray(nnz, np.int64)
        f = np.ascontiguousarray(fp, np.int64)
        admit = np.zeros(n, np.float64)
        start = np.zeros(n, np.float64)
        done = np.zeros(n, np.float64)
        lane = np.zeros(n, np.int32)
        mx = C.c_int64()
        ma = C.c_int32()
        p = lambda x: x.ctypes.data_as(C.c_void_p)
        nl = lib.sched_simulate(n, p(a), p(s), p(z), p(f), slots, C.c_uint64(budget), p(admit), p(start), p(done),
                                p(lane), C.byref(mx), C.byref(ma))
        run.start = start
        return nl, admit, done, lane, mx.value, ma.value
    return run


def _mix(count, seed):
    """Serving-like jobs: sizes from the per-job draws, Poisson arrivals at
    1000 jobs/s, service time proportional to size (fake clock)."""
    specs = I.serve_job_specs(count, seed)
    nnz, fp = [], []
    for spec, k, s in specs:
        if spec[0] == "grid":
            n = spec[1] ** 2
            m = 2 * (2 * spec[1] * (spec[1] - 1))
            w = False
        else:
            n = 1 << spec[1]
            m = int(0.8 * spec[2] * n * 2)  # about 80% of the R-MAT samples survive deduplication
            w = True
        nnz.append(m)
        fp.append(3 * (8 * (n + 1) + 4 * m * (2 if w else 1)) + 48 * n)
    arrival = I.arrivals(1000.0, count, seed + 7) * 1e3
    service = np.array([5.0 + x * 2e-6 for x in nnz])
    return arrival, service, np.array(nnz, np.int64), np.array(fp, np.int64)


def test_admission_respects_budget_and_order(sim):
    arrival, service, nnz, fp = _mix(400, 31)
    budget = int(4 * np.median(fp))
    budget = max(budget, int(fp.max()))
    nl, admit, done, lane, max_in_use, max_active = sim(arrival, service, nnz, fp, 64, budget)
    assert nl == 5
    assert (admit >= 0).all() and (done >= admit).all()     # every job admitted and finished
    assert max_in_use <= budget                              # never over the budget
    assert max_active <= 64
    assert (np.diff(admit) >= 0).all()                       # admission in submission order
    waited = admit - arrival
    assert (waited > 1e-9).sum() > 0                         # the budget binds: some jobs were held back
    # with no budget and slots to spare the same jobs are admitted on arrival
    _, admit2, _, _, _, _ = sim(arrival, service, nnz, fp, 1 << 20, 0)
    assert np.allclose(admit2, arrival)


def test_slots_bound_active_jobs(sim):
    arrival, service, nnz, fp = _mix(200, 32)
    for slots in (1, 2, 3, 8):
        nl, admit, done, lane, _, max_active = sim(arrival, service, nnz, fp, slots, 0)
        assert max_active <= slots and nl == min(slots, 5)
        if slots == 1:
            # one slot: strictly one job at a time, in order
            assert (admit[1:] >= done[:-1] - 1e-9).all()


def test_lanes_split_small_and_large(sim):
    arrival, service, nnz, fp = _mix(300, 33)
    nl, admit, done, lane, _, _ = sim(arrival, service, nnz, fp, 16, 0)
    start = sim.start
    small = nnz <= SMALL_NNZ
    assert (lane[small] == 0).all() and (start[small] == admit[small]).all()  # the batch lane takes them at once
    assert (lane[~small] >= 1).all() and (lane[~small] < nl).all()
    assert set(lane[~small].tolist()) == set(range(1, nl))                  # every single-job lane works
    # a single-job lane runs one job at a time, and large jobs start in admission order
    for l in range(1, nl):
        sel = np.where(lane == l)[0]
        order = np.argsort(start[sel])
        assert (start[sel][order][1:] >= done[sel][order][:-1] - 1e-9).all()
    big = np.where(~small)[0]
    assert (np.diff(start[big]) >= -1e-9).all()


def test_job_larger_than_budget_is_refused(sim):
    arrival = np.array([0.0, 1.0])
    fp = np.array([100, 1000], np.int64)
    rc, *_ = sim(arrival, np.array([1.0, 1.0]), np.array([10, 10], np.int64), fp, 4, 500)
    assert rc == -2  # the second job (index 1) cannot fit even alone


def test_large_job_is_not_starved(sim):
    """A large job that needs the whole budget waits only until the jobs
    admitted before it finish; later small jobs queue behind it."""
    arrival = np.arange(12, dtype=np.float64)
    fp = np.array([300] * 4 + [1000] + [100] * 7, np.int64)
    nnz = np.array([10] * 4 + [SMALL_NNZ * 4] + [10] * 7, np.int64)
    service = np.full(12, 50.0)
    nl, admit, done, lane, max_in_use, _ = sim(arrival, service, nnz, fp, 8, 1000)
    assert max_in_use <= 1000
    big = 4
    assert admit[big] == pytest.approx(max(done[:big]))     # right after the earlier jobs
    assert (admit[big + 1:] >= done[big] - 1e-9).all()        # the later ones wait for it
