import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and libimin.so")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def gpu():
    """Skip unless a GPU is present; then load the HIP library (fails loudly if unbuilt)."""
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_2302_13529_amd import binding
    binding.load()
    return binding
