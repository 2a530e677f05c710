"""CPU checks of bench.py's host logic: the algorithmic byte count of a gain
pass, the source check that keeps stored HBM traffic figures tied to the
kernel source they were taken on, and the refusal of more than one GPU."""
import hashlib
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_gain_bytes_full_records():
    # entries: 4 B id (+4 B weight); rows: 8 B offsets + 4 B part; vertices:
    # 4 B list entry (when listed) + 4 B part + 4 B lock + 8 B record
    assert bench.gain_bytes(10, 3, 4, weighted=True, listed=True) == 10 * 8 + 3 * 12 + 4 * 20
    assert bench.gain_bytes(10, 3, 4, weighted=False, listed=False) == 10 * 4 + 3 * 12 + 4 * 16


def test_gain_bytes_compact_records():
    # the 4-byte compact record per visited vertex, plus 4 B of F per vertex of X
    assert bench.gain_bytes(10, 3, 4, True, True, compact=True, in_x=2) == 10 * 8 + 3 * 12 + 4 * 16 + 2 * 4
    assert bench.gain_bytes(10, 3, 4, False, False, compact=True, in_x=0) == 10 * 4 + 3 * 12 + 4 * 12
    # |X| only counts where the compact records are written
    assert bench.gain_bytes(10, 3, 4, True, True, compact=False, in_x=5) == bench.gain_bytes(10, 3, 4, True, True)


def test_stored_traffic_needs_the_profiled_source(monkeypatch):
    src = os.path.join(ROOT, "paper_2304_13194_amd", "csrc", "jet_refine.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    rec = dict(fetch=100, write=20, fetch_factor=2.0, write_factor=1.0)
    monkeypatch.setitem(bench.TRAFFIC, "same_source", dict(rec, src_sha256=sha))
    monkeypatch.setitem(bench.TRAFFIC, "older_source", dict(rec, src_sha256="0" * 64))
    assert bench.measured_traffic("same_source")[0] == 120
    assert bench.measured_traffic("older_source") == (None, None)
    assert bench.measured_traffic("no_record") == (None, None)


def test_stored_traffic_records_are_complete():
    for name, t in bench.TRAFFIC.items():
        assert name in bench.WORKLOADS
        assert len(t["src_sha256"]) == 64 and t["fetch"] > 0 and t["write"] > 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
