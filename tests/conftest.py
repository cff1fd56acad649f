import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def c1_system():
    from synth.systems import make_config
    return make_config(1)


@pytest.fixture(scope="session")
def c1_oracle(c1_system):
    from oracle.pipeline import Oracle
    o = Oracle(c1_system)
    o.result = o.run(keep=True)
    return o
