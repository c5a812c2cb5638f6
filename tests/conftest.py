import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session", autouse=True)
def _built_cpu_libs():
    """The CPU-side shared objects (input generator, oracle) are built if absent."""
    import inputs
    import oracle
    if not os.path.exists(inputs._LIB):
        inputs.build(force=True)
    if not os.path.exists(oracle._LIB):
        oracle.build(force=True)
    yield
