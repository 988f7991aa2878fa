import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU statistical check")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def gctx():
    """mlmc context on cuda:0 (GPU tests only): fails loudly without the library."""
    import torch
    assert torch.cuda.is_available(), "GPU test needs a ROCm device"
    from paper_1505_00965_amd import mlmc
    ctx = mlmc.Context(0)
    yield ctx
    ctx.close()


@pytest.fixture(scope="session")
def torch_dev():
    import torch
    return torch.device("cuda:0")
