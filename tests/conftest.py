import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU cases of more than a few seconds (the larger degrees and "
                                       "paper rows of a pin whose cheaper cases always run); run with "
                                       "RZ_SLOW_TESTS=1")
    config.addinivalue_line("markers", "heavy: oracle builds of 20-80 s each; run only with RZ_HEAVY_TESTS=1")


def pytest_collection_modifyitems(config, items):
    heavy = bool(os.environ.get("RZ_HEAVY_TESTS"))
    slow = heavy or bool(os.environ.get("RZ_SLOW_TESTS"))
    skip_heavy = pytest.mark.skip(reason="oracle elements above p = 8 in 3D: set RZ_HEAVY_TESTS=1")
    skip_slow = pytest.mark.skip(reason="a larger case of a pin whose cheaper cases run: set RZ_SLOW_TESTS=1")
    for item in items:
        if "heavy" in item.keywords and not heavy:
            item.add_marker(skip_heavy)
        elif "slow" in item.keywords and "gpu" not in item.keywords and not slow:
            item.add_marker(skip_slow)
