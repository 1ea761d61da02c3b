import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


def pytest_collection_modifyitems(config, items):
    # GPU tests fail loudly (not skip) when the device or the HIP library is
    # missing; they are deselected on CPU-only runs with -m "not gpu".
    pass


@pytest.fixture(scope="session")
def repo_root():
    return ROOT
