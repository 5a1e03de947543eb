import functools
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")


@functools.lru_cache(maxsize=None)
def workload(k, **kw):
    from paper_2608_12691_amd import systems
    return systems.make_config(k, **kw)


@pytest.fixture(scope="session")
def cfg1():
    return workload(1)


@pytest.fixture(scope="session")
def cfg2():
    return workload(2)
