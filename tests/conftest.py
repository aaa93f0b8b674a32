import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built libace.so")
    config.addinivalue_line("markers", "slow: large CPU case")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def need_gpu():
    if not gpu_available():
        pytest.fail("GPU test run without a visible GPU")


# Launch tunings the GPU parity tests run under: the library's own defaults and
# the autotuned one saved for the device (the one the benchmarks install).
# They reach different branches: persistent tiles per atomic grab, the
# in-order graph's passes over its grid, the batch size from which an open
# call bins by block count.
TUNINGS = ["library-default", "saved"]


def use_tuning(ace, which: str) -> dict:
    from paper_2603_10242_amd import autotune
    ace.set_tuning(**ace.default_tuning())
    if which == "saved" and autotune.apply_saved() is None:
        pytest.fail("no saved launch tuning for this device")
    return ace.get_tuning()
