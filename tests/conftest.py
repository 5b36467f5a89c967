import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU; parity tests against the CPU oracle")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def oracle():
    from oracle import oracle as O
    O.build()
    return O


@pytest.fixture(scope="session")
def gpu():
    """The HIP binding; fails (never skips) when no GPU is visible."""
    import torch
    assert torch.cuda.is_available(), "gpu-marked test run without a visible GPU"
    from paper_1705_06149_amd import nsp
    nsp.lib()
    return nsp
