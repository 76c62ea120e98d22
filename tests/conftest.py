import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running (exhaustive CPU pins, full-size GPU workloads)")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import build as obuild
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        obuild.build()
    from oracle import oracle
    return oracle
