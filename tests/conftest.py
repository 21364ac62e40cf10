import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")
    config.addinivalue_line("markers", "slow: long-running CPU oracle case")


@pytest.fixture(scope="module")
def hps():
    """The HIP library's binding (GPU tests only; importing it loads the built
    library and fails loudly when it is missing)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_00735_amd import hps as _hps
    return _hps


@pytest.fixture(scope="module")
def ctx(hps):
    return hps.Context()
