import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def orc():
    """The CPU FP64 oracle (built once per session)."""
    from oracle import oracle as O
    O.build(force=not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")))
    return O


@pytest.fixture(scope="session")
def pr():
    from paper_1109_3577_amd import problems
    return problems
