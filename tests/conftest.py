import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test taking more than a few seconds")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def bfi():
    import paper_1803_07560_amd as bfi_mod
    bfi_mod.load()
    return bfi_mod


@pytest.fixture(scope="session")
def ctx(bfi):
    """A bfi context on device 0 (GPU tests only)."""
    c = bfi.bfi_context_create(0)
    yield c
    bfi.bfi_context_destroy(c)
