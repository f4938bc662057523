import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the HIP library")


def golden_path(name):
    return os.path.join(GOLDEN, name)


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def abm():
    """The HIP library binding; builds libabm.so here if it is absent."""
    import paper_2508_16508_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        from paper_2508_16508_amd import _build
        _build.build()
    pkg.lib()
    return pkg
