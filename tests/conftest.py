import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")
    config.addinivalue_line("markers", "slow: long CPU run of the oracle; opt in with -m slow")


def pytest_collection_modifyitems(config, items):
    # slow oracle runs are opt-in: skip them unless the -m expression names them
    expr = config.getoption("-m") or ""
    if "slow" in expr:
        return
    skip = pytest.mark.skip(reason="slow oracle run; select with -m slow")
    for it in items:
        if "slow" in it.keywords:
            it.add_marker(skip)
