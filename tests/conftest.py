import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-only check")


@pytest.fixture(scope="session")
def oracle():
    import oracle as _oracle
    _oracle.build()
    return _oracle


@pytest.fixture(scope="module")
def km():
    """The package's shared context on cuda:0.  At the end of every module
    the context is synchronised, which reports a persistent Lloyd launch of
    that module whose barrier gave up."""
    import paper_1412_1947_amd as pkg
    ctx = pkg.context(0)
    yield ctx
    ctx.synchronize()
