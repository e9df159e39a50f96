import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test taking more than a few seconds")
    # (re)build the C oracle here, at session start, before any test touches
    # the GPU: the oracle's loader itself never compiles
    import oracle
    oracle.build(force=False)


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle
