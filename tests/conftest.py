import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    import gpu_util

    gpu_util.CAPTURE_MANAGER = config.pluginmanager.getplugin("capturemanager")
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: full-size workloads (minutes of CPU)")


def pytest_collection_modifyitems(config, items):
    # GPU tests run in file order; keep them grouped so a failure names the step.
    pass


@pytest.fixture(scope="session")
def golden_dir():
    return os.path.join(HERE, "golden")
