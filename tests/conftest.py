import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _built_helpers():
    # the oracle and the node-set helper are plain C built with gcc; build
    # them once if a fresh checkout has no shared objects yet
    import nodesets
    import oracle.build
    if not os.path.exists(oracle.oracle.LIB_PATH):
        oracle.build.build()
    if not os.path.exists(nodesets._SO):
        nodesets.build()
    yield
