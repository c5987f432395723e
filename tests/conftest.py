import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")


@pytest.fixture(scope="session", autouse=True)
def _host_libs():
    """Compile the host-only helpers (stroke builder, oracle) if missing."""
    import canvasgen
    from oracle import oracle
    canvasgen.build_lib(force=False)
    oracle.build(force=False)
