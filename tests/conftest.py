import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def grf():
    """The HIP library binding; GPU tests only."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_02670_amd import grf as _grf

    _grf.load()
    return _grf
