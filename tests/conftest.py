import os
import pathlib
import sys

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))


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
