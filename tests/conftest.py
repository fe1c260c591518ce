import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle():
    import oracle as o
    o.build(force=False)
    return o


@pytest.fixture(autouse=True)
def _hip_notes(request):
    """Around every GPU test: HIP errors that no library call could return
    to its caller. A failure on one of the library's own release paths fails
    the test; an error some other HIP call left pending (found and cleared by
    the library before a launch) is reported as a warning naming the test."""
    if request.node.get_closest_marker("gpu") is None:
        yield
        return
    from paper_1609_01257_amd import rngx
    rngx.hip_notes(clear=True)
    yield
    notes = rngx.hip_notes(clear=True)
    if notes["stray"]:
        import warnings
        warnings.warn("HIP errors left pending by other calls during %s: %s"
                      % (request.node.nodeid, notes["notes"]))
    if notes["released"]:
        pytest.fail("library release paths failed: %s" % notes["notes"], pytrace=False)
