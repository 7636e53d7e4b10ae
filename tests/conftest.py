import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")
    # The CPU-only selection runs the oracle on small matrices: a few BLAS
    # threads are as fast as many there, and they keep OpenBLAS's spinning
    # threads from stalling the suite when other work shares the host's
    # cores.  Set before the test modules (and numpy) are imported.
    if "not gpu" in (config.getoption("markexpr", "") or ""):
        os.environ.setdefault("OPENBLAS_NUM_THREADS", "4")
