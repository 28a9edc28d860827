import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    from tests import progress
    progress._config = config


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    from oracle import oracle as O
    if not os.path.exists(O.LIB_PATH):
        O.build()
    yield
