import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def lgf_gpu():
    """The GPU binding; the test fails loudly if the HIP library is absent."""
    import torch

    if not torch.cuda.is_available():
        pytest.fail("gpu test run without a visible GPU")
    import paper_1301_3460_amd as lgf

    lgf.load()  # raises if liblgf.so is missing
    return lgf
