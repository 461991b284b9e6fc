import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def oracle():
    import oracle as O
    O.lib()
    return O


@pytest.fixture(scope="session")
def msst():
    """The HIP library binding; a GPU test fails (never skips) without it."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_2011_03082_amd as M
    M.lib()
    return M


def announce(msg):
    """Names the GPU case about to run, flushed, so a crash log shows it."""
    print(f"[gpu-case] {msg}", flush=True)
