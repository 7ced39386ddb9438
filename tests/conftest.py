import os
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def _ensure_built():
    """Build libstmg.so once if it is missing (the tests load what is built)."""
    lib = ROOT / "paper_2505_10168_amd" / "_lib" / "libstmg.so"
    if lib.exists() or not (ROOT / "paper_2505_10168_amd" / "build.py").exists():
        return
    from paper_2505_10168_amd.build import build
    build(verbose=False)


_ensure_built()


@pytest.fixture(scope="session")
def cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    return torch.device("cuda:0")


@pytest.fixture(autouse=True)
def _announce(request):
    # name the case before any GPU work so a fault can be traced to it
    if request.node.get_closest_marker("gpu") is not None:
        print(f"\n[case] {request.node.nodeid}", flush=True)
    yield
