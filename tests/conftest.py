import os
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def _ensure_built():
    lib = ROOT / "paper_2104_10523_amd" / "libtn.so"
    if not lib.exists():
        from paper_2104_10523_amd.build import build
        build()


_ensure_built()


@pytest.fixture(scope="session")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no GPU is visible")
    return torch.device("cuda:0")


@pytest.fixture(scope="session")
def workspace(gpu):
    import torch
    import paper_2104_10523_amd as tn
    buf = torch.empty(1 << 30, dtype=torch.uint8, device=gpu)
    tn.tn_set_workspace(buf)
    yield buf
    tn.tn_set_workspace(None)
