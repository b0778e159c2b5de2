import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU oracle check")


@pytest.fixture(scope="session")
def gpu_ctx():
    """Library context on cuda:0 bound to torch's current stream (GPU tests only)."""
    import torch
    from paper_1811_06797_amd import iga
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.init()
    stream = torch.cuda.current_stream().cuda_stream
    ctx = iga.ctx_create(0, stream)
    yield ctx
    torch.cuda.synchronize()
    iga.ctx_destroy(ctx)
