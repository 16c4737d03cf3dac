import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def tk():
    """The GPU library binding; GPU tests need it loaded (no fallback)."""
    if not gpu_available():
        pytest.skip("no GPU")
    import paper_1805_07801_amd as tkmod
    tkmod.load()
    return tkmod


@pytest.fixture(scope="session")
def band512():
    """The 512^3 band-filling solenoidal field (every kept mode O(1), unit energy, FP64,
    from the seed-2 noise), built once by the oracle and shared by the full-size tests."""
    import synth
    from oracle import init as oinit
    return oinit.band_filling(synth.gaussian_field((3, 512, 512, 512), 2))
