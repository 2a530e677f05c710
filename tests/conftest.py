import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger sizes; still CPU-only")


def graph_from_edges(n, edges, vwgt=None):
    from paper_2304_13194_amd.inputs import csr_from_edges
    e = np.array(edges, dtype=np.int64).reshape(-1, 3)
    return csr_from_edges(n, e[:, 0], e[:, 1], e[:, 2].astype(np.int32),
                          vwgt=None if vwgt is None else np.array(vwgt, np.int32))


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import oracle
    oracle.lib()
    return oracle
