import os
import sys
import warnings

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")
    warnings.filterwarnings("ignore", message=".*roundoff error.*")
    warnings.filterwarnings("ignore", message=".*algorithm does not converge.*")


@pytest.fixture(scope="session")
def oracle():
    from oracle import glo
    glo.lib()
    return glo


def _gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def gpu_lib():
    """The built HIP library, loaded through its binding.  A GPU test that
    reaches this fixture on a host without a GPU fails loudly rather than
    falling back to anything."""
    if not _gpu_available():
        pytest.fail("GPU test collected on a host without a visible GPU")
    from paper_2410_05408_amd import gl
    return gl
