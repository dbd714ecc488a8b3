import os
import sys

# GPU tests run with poisoned workspaces: a kernel that reads scratch memory
# it did not write sees NaN and the parity check fails.
os.environ.setdefault("DDPPO_POISON_WS", "1")

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def P():
    """The library's Python binding (GPU tests)."""
    import torch
    import paper_1911_00357_amd as P
    assert torch.cuda.is_available()
    return P
