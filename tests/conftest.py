import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running test (full-size inputs)")


@pytest.fixture
def progress(request):
    """say(msg): a progress line written past pytest's output capture, so a
    long phase of a test (a full-size oracle run) shows that it is alive."""
    import time
    capman = request.config.pluginmanager.getplugin("capturemanager")

    def say(msg):
        with capman.global_and_fixture_disabled():
            sys.stderr.write(f"[{request.node.name} {time.strftime('%H:%M:%S')}] {msg}\n")
            sys.stderr.flush()
    return say


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP path through its C ABI; skips when no GPU is visible."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2206_09960_amd import api
    api.load()  # raises if the HIP library is missing
    return api
