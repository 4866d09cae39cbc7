import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU run (oracle physics at larger sizes)")


@pytest.fixture(scope="session")
def gpu():
    """The HIP binding with a GPU present; GPU tests fail loudly if the library is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2506_21804_amd as lbm
    lbm.load()  # raises if the built HIP library is missing
    return lbm
