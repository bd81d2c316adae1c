import os
import sys

# The oracle's dot products go through BLAS; with several threads the
# summation order (and so the last bits of every reduction, which long
# Krylov trajectories amplify) depends on the thread count.  One thread
# makes every oracle result reproducible on any host.
for _var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_var] = "1"

import pytest  # noqa: E402
from threadpoolctl import threadpool_limits  # noqa: E402

threadpool_limits(1)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def golden_dir():
    return os.path.join(ROOT, "tests", "golden")
