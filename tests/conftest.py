import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build()
    threads = int(os.environ.get("ORACLE_THREADS", "0")) or min(16, os.cpu_count() or 1)
    oracle.set_threads(threads)
    return oracle


@pytest.fixture(scope="session")
def inputs_mod():
    from paper_2208_01260_amd import inputs
    return inputs
