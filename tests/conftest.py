import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


def pytest_collection_modifyitems(config, items):
    # Oracle solves marked slow (minutes each on the CPU) run only with
    # BMG_SLOW_TESTS=1, so that the default CPU suite takes a few minutes.
    if not os.environ.get("BMG_SLOW_TESTS"):
        skip_slow = pytest.mark.skip(reason="slow oracle solve; set BMG_SLOW_TESTS=1 to run")
        for it in items:
            if "slow" in it.keywords:
                it.add_marker(skip_slow)
    # GPU tests are skipped (not failed) when no GPU is visible, so that the
    # CPU suite stays green; on a machine with a GPU they run and must pass.
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)
