import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def rng():
    import numpy as np
    return np.random.default_rng(20240606)


@pytest.fixture(scope="session", autouse=True)
def _library_built():
    """Build libptycho.so in-tree once if it is missing (a fresh checkout)."""
    import importlib
    lib = os.path.join(ROOT, "paper_2406_06640_amd", "_lib", "libptycho.so")
    if not os.path.exists(lib):
        build = importlib.import_module("paper_2406_06640_amd.build")
        build.build()
    yield
