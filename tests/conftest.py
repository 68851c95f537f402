import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI on the device)")
    config.addinivalue_line("markers", "slow: long CPU run (oracle physics checks)")


def pytest_collection_modifyitems(config, items):
    # order: CPU tests first, GPU tests after, within a file keep definition order
    items.sort(key=lambda it: 1 if it.get_closest_marker("gpu") else 0)
