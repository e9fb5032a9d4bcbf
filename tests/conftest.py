import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI on the device)")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build()
    return oracle


@pytest.fixture(scope="session")
def nlth_mod():
    """The ctypes binding; builds libnlth.so only if it is not built yet."""
    from paper_2604_02755_amd import nlth
    if not os.path.exists(nlth.LIB_PATH):
        from paper_2604_02755_amd import build
        build.build()
    nlth.lib()
    return nlth


@pytest.fixture(scope="session")
def gpu_ctx(nlth_mod):
    ctx = nlth_mod.Context(0, use_torch_stream=False)
    yield ctx
    ctx.close()
