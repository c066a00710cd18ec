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
def oracle_lib():
    import oracle
    oracle.build_oracle(force=False)
    return oracle.load_oracle()


@pytest.fixture(autouse=True)
def _announce(request):
    # name the case before it runs, so a stall can be attributed
    print(f"\n[start] {request.node.nodeid}", flush=True)
    yield
