import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session", autouse=True)
def built_library():
    """Build the HIP library in-tree once if it is not there (hipcc cross-compiles without a GPU)."""
    from paper_1905_02803_amd import LIB_PATH

    if not os.path.exists(LIB_PATH):
        from paper_1905_02803_amd import build

        build.build()
