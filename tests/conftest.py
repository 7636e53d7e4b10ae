import os
import sys

# The oracle's matrices in the tests are small: a few BLAS threads are as
# fast as many, and they avoid OpenBLAS's spin-waiting threads stalling the
# suite when other work shares the host's cores.  Set before numpy loads.
os.environ.setdefault("OPENBLAS_NUM_THREADS", "4")

import pytest  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")
