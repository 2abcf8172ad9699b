import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built HIP library")
    expr = config.getoption("markexpr", default="") or ""
    if "gpu" in expr and "not gpu" not in expr:
        # the first torch import on a fresh machine can take minutes: do it
        # before any per-test time limit starts
        import torch  # noqa: F401


@pytest.fixture(autouse=True)
def _gpu_required(request):
    if request.node.get_closest_marker("gpu"):
        import torch
        if not torch.cuda.is_available():
            pytest.fail("GPU test on a machine without a visible GPU")
