import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built device library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


# the oracle works in float64; make stray torch.tensor(python_float) calls in
# tests float64 too
import torch  # noqa: E402

torch.set_default_dtype(torch.float64)


def pytest_collection_modifyitems(config, items):
    """GPU tests are skipped (not failed) where no GPU is visible."""
    if torch.cuda.is_available():
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)
