import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: large inputs (seconds to minutes)")


@pytest.fixture(scope="session", autouse=True)
def _built_host_libs():
    """Compile the two host-side C helpers (input generators, oracle) once."""
    import graphgen
    import oracle
    if not os.path.exists(graphgen._LIB_PATH):
        graphgen.build()
    if not os.path.exists(oracle._LIB_PATH):
        oracle.build()
    yield
