"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle's C source is built with gcc's host sanitizers and driven, in a
child process that preloads the ASan runtime, through every exported call:
a refinement loop, single Jetlp and rebalancing steps, matching, two-hop
matching, contraction, the graph-growing start and full multilevel
partitions, including empty, isolated-vertex and k = 1 cases. Any invalid
access, overflow of a signed integer or other undefined behaviour aborts the
child with a report, and the test fails with that report.
"""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "jet_oracle.c")

DRIVER = textwrap.dedent("""
    import sys
    import numpy as np
    sys.path.insert(0, sys.argv[1])
    from oracle import oracle as O
    from paper_2304_13194_amd import inputs as I
    from tests.conftest import graph_from_edges
    with O.use_library(sys.argv[2]):
        cases = [
            (I.grid2d(17, 13), 4),
            (I.stencil27(6, 5, 4), 5),
            (I.small_random_graph(60, 0.08, 9, wmax=7, vwmax=4), 3),
            (I.rmat(9, 4, 3), 8),
            (graph_from_edges(7, [(0, 1, 2), (1, 2, 1)]), 2),      # isolated vertices
            (graph_from_edges(201, [(0, i, 1) for i in range(1, 201)]), 2),  # a star
        ]
        for g, k in cases:
            P = I.random_partition(g.n, k, 5)
            O.refine(g, P, k, seed=1)
            O.refine(g, P, 1, seed=1)
            O.jetlp(g, P, np.zeros(g.n, np.uint8), k)
            O.rebalance(g, np.zeros(g.n, np.int32), 2, 0, k, seed=2)
            O.rebalance(g, np.zeros(g.n, np.int32), 3, 1, k, seed=2)
            nc, cmap = O.hem_map(g, 0, 7)
            O.contract(g, cmap, nc)
            O.hem_map(g, 1, 7, two_hop=True)
            O.bfs_part(g, k)
            O.partition(g, k, seed=4)
            O.partition(g, k, seed=4, flags=O.F_TWO_HOP | O.F_BFS_START)
        e = graph_from_edges(0, [])
        O.refine(e, np.zeros(0, np.int32), 3)
        O.partition(e, 3)
    print("sanitized oracle ok", flush=True)
""")


def test_oracle_under_asan_and_ubsan(tmp_path):
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("gcc's ASan runtime is not installed")
    so = tmp_path / "libjetoracle_san.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=gnu11", "-shared", "-fPIC", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", str(so), SRC])
    drv = tmp_path / "drive.py"
    drv.write_text(DRIVER)
    env = dict(os.environ, LD_PRELOAD=libasan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, str(drv), ROOT, str(so)], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0 and "sanitized oracle ok" in r.stdout, (r.stdout[-2000:] + r.stderr[-6000:])
