import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def oracle_beta(g, c):
    """beta = c / lambda_max(A) with the oracle's own lambda_max: tests pick
    beta on their side and hand the same value to the index build and to the
    oracle, so no oracle input comes from the library."""
    import oracle
    return c / oracle.lambda_max(oracle.csr_matrix(g.n, g.row_ptr, g.col))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: large workload, minutes of host time")


def pytest_collection_modifyitems(config, items):
    # GPU tests need a visible device; on a host without one they are
    # skipped (select them with -m gpu).
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:
        have_gpu = False
    if have_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)
