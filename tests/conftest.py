import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running statistical check")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    from oracle import build as ob
    ob.build()
    return oracle


def _gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def smc_gpu():
    """The HIP library bound through the Python binding; skips without a GPU."""
    if not _gpu_available():
        pytest.skip("no GPU visible")
    import paper_1107_5463_amd as smc
    smc.load_library()
    return smc
