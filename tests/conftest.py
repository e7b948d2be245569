import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


def pytest_collection_modifyitems(config, items):
    # GPU tests are ordered after CPU tests; the no-allocation test file last.
    items.sort(key=lambda it: (1 if it.get_closest_marker("gpu") else 0,
                               1 if "test_zz_" in it.nodeid else 0))
