import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")
for _p in (ROOT, TESTS):          # the oracle pool's workers import tests/oracle_pool.py by name
    if _p not in sys.path:
        sys.path.insert(0, _p)

GOLDEN = os.path.join(ROOT, "tests", "golden")


# Worker processes for the full-size oracle comparisons of the GPU tests.
# They are forked here, before any test (or test-module import) touches the
# GPU, and they run only the NumPy oracle: no process is ever forked or
# exec'd from one that has initialised the GPU.
_POOL = None


def _gpu_session(config):
    m = (config.getoption("markexpr", "") or "").replace(" ", "")
    return "gpu" in m and "notgpu" not in m


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")
    global _POOL
    if _gpu_session(config) and os.environ.get("BICOP_ORACLE_WORKERS", "") != "0":
        from oracle_pool import OraclePool
        workers = int(os.environ.get("BICOP_ORACLE_WORKERS", "0")) or min(16, os.cpu_count() or 1)
        _POOL = OraclePool(workers)


def pytest_unconfigure(config):
    global _POOL
    if _POOL is not None:
        _POOL.close()
        _POOL = None


@pytest.fixture(scope="session")
def oracle_pool():
    """The forked oracle workers of a GPU session, or None (chunks then run in-process)."""
    return _POOL


def read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows


@pytest.fixture
def golden():
    return read_golden
