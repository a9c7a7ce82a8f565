import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

try:  # small dense matrices: BLAS threading only adds overhead.  The limit
    # applies to the BLAS libraries loaded when it is set, so load them first.
    import numpy.linalg  # noqa: F401
    import scipy.fft  # noqa: F401
    import scipy.linalg  # noqa: F401
    import threadpoolctl

    threadpoolctl.threadpool_limits(1, user_api="blas")
except Exception:  # pragma: no cover
    pass

# the oracle's FFT workers: the cores this process may run on (at most 16)
_CORES = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
from oracle import operators as _op  # noqa: E402

_op._WORKERS = max(1, min(_CORES, 16))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_collection_modifyitems(config, items):
    have_gpu = False
    try:
        import torch

        have_gpu = torch.cuda.is_available()
    except Exception:
        have_gpu = False
    if have_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)
