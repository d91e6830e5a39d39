import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def ref():
    """The FP64 CPU oracle (built on first use if nothing is built).  Its
    OpenMP loops have no reductions, so the thread count changes only the
    speed; half the cores available (the host's, capped by OMP_NUM_THREADS)
    keep its many short parallel loops (1D) from waiting on threads that the
    host is using for something else."""
    import oracle

    n = os.cpu_count() or 2
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    oracle.lib().dgref_set_threads(max(1, n // 2))
    return oracle


def gpu_available() -> bool:
    try:
        import torch

        return torch.cuda.is_available()
    except Exception:
        return False
