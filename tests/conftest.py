import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The oracle's dense LAPACK calls are small: run them on one thread.  A threaded OpenBLAS has twice
# reported an exact zero pivot (the same 36 x 36 solve, condition number ~150) on a 16-thread host,
# which no single-threaded run reproduces.
try:
    from threadpoolctl import threadpool_limits
    _BLAS_LIMIT = threadpool_limits(limits=1, user_api="blas")
except ImportError:          # threadpoolctl missing: keep the library defaults
    _BLAS_LIMIT = None


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU cases (still minutes at most)")
