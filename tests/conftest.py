import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def rng():
    import numpy as np
    return np.random.default_rng(12345)


@pytest.fixture(scope="session")
def built_lib():
    """The in-tree HIP library; built here (hipcc cross-compiles for gfx950) only if absent."""
    from paper_1209_5942_amd import tmqcd
    if not os.path.exists(tmqcd.LIB_PATH):
        from paper_1209_5942_amd import build
        build.build()
    return tmqcd.LIB_PATH
