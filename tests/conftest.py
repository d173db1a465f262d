import os
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")
    # the library's autotune cache goes to a file of this session, not to the
    # user's cache directory
    if "TZ_TUNE_CACHE" not in os.environ:
        os.environ["TZ_TUNE_CACHE"] = os.path.join(tempfile.mkdtemp(prefix="tz_tune_"), "tune.json")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle
