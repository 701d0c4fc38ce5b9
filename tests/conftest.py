import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    # progress lines of long tests reach the terminal under output capture too
    import gpu_helpers
    gpu_helpers.CAPTURE_MANAGER = config.pluginmanager.getplugin("capturemanager")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def inputs_mod():
    from paper_1803_03922_amd import inputs
    inputs.build(force=False)
    return inputs
