import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU oracle case")


@pytest.fixture(scope="session")
def gpu_available():
    import torch
    return torch.cuda.is_available()


@pytest.fixture(scope="session")
def torch_cuda():
    """torch with the library loaded; skips without a GPU."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_02925_amd import lowrank
    lowrank.load_library()
    return torch
