import os
import sys
from pathlib import Path

import numpy as np
import pytest

ROOT = Path(__file__).resolve().parent.parent
sys.path.insert(0, str(ROOT))

# The oracle pins call dense LAPACK; with every core's worth of BLAS threads they
# spin against any other process on the host and slow down by an order of magnitude,
# so the session keeps the BLAS pool small.
try:
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=max(1, min(4, (os.cpu_count() or 2) // 2)))
except ImportError:
    pass


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a HIP device (MI355X); runs the HIP library")
    config.addinivalue_line("markers", "slow: CPU test taking more than a few seconds")


def _gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if _gpu_available():
        return
    skip = pytest.mark.skip(reason="no HIP device")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


@pytest.fixture(scope="session")
def sscg():
    import paper_1004_0292_amd as S
    S.lib()
    return S


def step(msg):
    """Name the case before a GPU step (printed and flushed)."""
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="session")
def cfg1_dense():
    """The 4^4 workload's explicit matrix and its dense eigen-decomposition, computed
    once per session (several oracle pins compare against it)."""
    import synth
    from oracle import wilson
    w = synth.CONFIGS["wilson4_fp64"]
    U = w.gauge()
    A = wilson.hermitian_wilson(U, w.dims, w.kappa)
    lam, W = np.linalg.eigh(A.toarray())
    return U, A, lam, W
