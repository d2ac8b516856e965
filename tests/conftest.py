import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session", autouse=True)
def _built_cpu_libs():
    """The oracle and the scene renderer are plain C; build them once if they
    are missing (the GPU library is built by __graft_entry__.build())."""
    import oracle
    import scenegen
    oracle.build(force=False)
    scenegen.build(force=False)
