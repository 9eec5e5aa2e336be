import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI on the device)")
    config.addinivalue_line("markers", "slow: larger CPU-only cases")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build()
    return oracle.lib()


@pytest.fixture(scope="session")
def gpu():
    """The loaded GPU library; fails (does not skip) when there is no device."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no HIP device is visible")
    import paper_1508_03619_amd as gb
    gb.load()
    return gb


@pytest.fixture(autouse=True)
def _device_status(request):
    """After every GPU test: no search queued on the current stream may have
    failed on the device unnoticed (gap_stream_status)."""
    yield
    if request.node.get_closest_marker("gpu") is None:
        return
    import torch
    if not torch.cuda.is_available():
        return
    from paper_1508_03619_amd import gapbfs
    gapbfs.stream_status()
