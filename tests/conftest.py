import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

_POOL = {}


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "oracle_pool: runs the FP64 oracle in worker processes")


@pytest.hookimpl(trylast=True)
def pytest_collection_modifyitems(session, config, items):
    # The oracle's worker processes are forked here, after collection and
    # before any test has touched the GPU, and only when a selected test
    # asks for them.
    if any(item.get_closest_marker("oracle_pool") for item in items):
        from oracle import pool
        _POOL["pool"] = pool.Pool()


def pytest_unconfigure(config):
    p = _POOL.pop("pool", None)
    if p is not None:
        p.terminate()
        p.join()


@pytest.fixture(scope="session")
def oracle_pool():
    """A pool of oracle worker processes (forked before any GPU call)."""
    p = _POOL.get("pool")
    if p is None:
        pytest.fail("the test needs the oracle_pool marker")
    return p


def read_golden(name):
    """key = value lines of a tests/golden fixture (comments start with #)."""
    import numpy as np
    out = {}
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            k, v = line.split("=", 1)
            out[k.strip()] = np.array([float(x) for x in v.split()], dtype=np.float64)
    return out
