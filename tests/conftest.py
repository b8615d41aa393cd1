import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")
    # Tests that hand torch device buffers to the library need torch's GPU runtime
    # initialised before the library first touches the GPU (as bench.py and smoke()
    # do): torch reports no GPU when its runtime starts second in the process.
    if "gpu" in (config.getoption("-m", default="") or ""):
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()


def pytest_collection_modifyitems(config, items):
    # keep GPU tests grouped after CPU tests inside one run
    items.sort(key=lambda it: 1 if it.get_closest_marker("gpu") else 0)
