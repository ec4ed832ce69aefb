import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: full-size inputs (seconds to minutes)")


def pytest_collection_modifyitems(config, items):
    # every test file named test_gpu_* needs the GPU
    for it in items:
        if os.path.basename(str(it.fspath)).startswith("test_gpu"):
            it.add_marker(pytest.mark.gpu)
