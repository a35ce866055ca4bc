import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def gpu():
    """The torch device for GPU tests; fails (not skips) when the GPU or the
    HIP library is missing, so a GPU run never passes on a fallback."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("gpu-marked test run without a visible GPU")
    import paper_2603_20889_amd as q
    q.load()   # raises when libqless.so is missing or not loadable
    return torch.device("cuda:0")
