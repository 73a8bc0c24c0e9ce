import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: oracle cases that take tens of seconds on the CPU")


def pytest_collection_modifyitems(config, items):
    # order: CPU tests first, GPU tests after, so a GPU failure hides no CPU result
    items.sort(key=lambda it: 1 if it.get_closest_marker("gpu") else 0)
