import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session", autouse=True)
def _native_test_libs():
    """The oracle and the scene renderer are plain C; build them if absent."""
    import oracle
    import synth
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build(force=False)
    if not os.path.exists(synth.LIB_PATH):
        synth.build(force=False)
    yield


@pytest.fixture(scope="session")
def box_room():
    import synth
    return synth.workload("box_room_256", seed=0)
