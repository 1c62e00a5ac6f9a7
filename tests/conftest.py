import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU oracle run")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def cm():
    """The cmlb binding; builds libcmlb.so only if it is absent."""
    from paper_1808_04406_amd import cmlb
    if not os.path.exists(cmlb.LIB_PATH):
        from paper_1808_04406_amd import build
        build.build()
    cmlb.lib()
    return cmlb
