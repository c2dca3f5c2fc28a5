import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def O():
    """The oracle package (built on first use)."""
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(autouse=True)
def _announce(request):
    """Name each test, flushed, before it runs (a hang then names its case)."""
    line = f"[start] {request.node.nodeid}\n"
    sys.stderr.write(line)
    sys.stderr.flush()
    out = os.environ.get("PPM_TEST_PROGRESS")   # optional file that mirrors these lines
    if out:
        with open(out, "a") as f:
            f.write(line)
    yield
