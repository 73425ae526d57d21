import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build()
    return oracle


@pytest.fixture(scope="session")
def sb():
    """The GPU library binding on cuda:0 (GPU tests only)."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2108_02025_amd as sbmod
    sbmod.load()  # raises if the HIP library is not built
    return sbmod
