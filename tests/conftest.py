import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running statistical test")


@pytest.fixture(scope="session")
def paper_constants():
    import json
    with open(os.path.join(ROOT, "tests", "golden", "paper_constants.json")) as f:
        return json.load(f)


@pytest.fixture(scope="session", autouse=True)
def _oracle_threads():
    """The oracle's per-domain loops on up to 16 host threads (the trajectory is
    bit-identical for every thread count; only the full-size comparisons need
    the speed)."""
    import oracle
    oracle.set_threads(min(16, os.cpu_count() or 1))
    yield
    oracle.set_threads(1)


@pytest.fixture(scope="session", autouse=True)
def _release_device_objects():
    """After the last test: drop the library's cached batch workspaces and wait
    for the device, so nothing of the library is freed by exit-time handlers."""
    yield
    import sys as _sys
    mod = _sys.modules.get("paper_1005_4713_amd.spkmc")
    if mod is not None:
        import gc
        gc.collect()
        mod.release_cached()
