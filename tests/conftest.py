import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")
    config.addinivalue_line("markers", "heavy: oracle builds of 20-80 s each; run only with RZ_HEAVY_TESTS=1")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("RZ_HEAVY_TESTS"):
        return
    skip = pytest.mark.skip(reason="oracle elements above p = 8 in 3D: set RZ_HEAVY_TESTS=1")
    for item in items:
        if "heavy" in item.keywords:
            item.add_marker(skip)
