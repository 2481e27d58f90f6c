import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-side oracle run")


@pytest.fixture(scope="session")
def oracle_omp(tmp_path_factory):
    """The oracle's sources built -O3 -march=native with OpenMP (the plain
    build's bits with any number of threads, tests/test_abi.py), for the
    parity runs of the larger workloads; uses every thread OpenMP is given."""
    import oracle
    so = oracle.build_baseline(str(tmp_path_factory.mktemp("oracle_omp") / "liboracle_omp.so"))
    oracle.set_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), so)
    return so
