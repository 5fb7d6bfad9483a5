import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running")


@pytest.fixture(scope="session")
def gpu():
    """The HIP library bound to cuda:0; fails loudly if either is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    import paper_1312_6838_amd as g
    g.load()
    return g


def pytest_runtest_logstart(nodeid, location):
    # name the case before it touches the GPU, so a run that dies still says which
    print(f"\n[start] {nodeid}", flush=True)
