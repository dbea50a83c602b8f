import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library on a machine with an MI355X; fails loudly when it is not built."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    import paper_0809_1906_amd as bcgpu
    import paper_0809_1906_amd.binding  # noqa: F401
    bcgpu.load()  # raises if the shared library is missing
    return bcgpu
