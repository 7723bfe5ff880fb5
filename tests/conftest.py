import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test taking more than a few seconds")


@pytest.fixture(scope="session", autouse=True)
def _built_helpers():
    """The generator and oracle libraries are plain C; build them if absent."""
    import graphgen
    import oracle
    graphgen.build(force=False)
    oracle.build(force=False)
