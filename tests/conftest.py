import os
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# launch shapes the tests tune go to a file of the test session, not to the
# user's tuning cache that later processes (a benchmark) would read
os.environ.setdefault("PRECODE_TUNE_CACHE", os.path.join(tempfile.mkdtemp(prefix="precode_tests_"), "tune.txt"))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle

    oracle.build(force=False)
    return oracle
