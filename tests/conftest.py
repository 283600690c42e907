import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU test (runs only when -m selects 'slow')")


def pytest_collection_modifyitems(config, items):
    """Slow tests run only when the marker expression names them (-m slow)."""
    if "slow" in (config.getoption("markexpr") or ""):
        return
    skip = pytest.mark.skip(reason="slow: select with -m slow")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)


KEY_SEED = 0x5EED0001


@pytest.fixture(scope="session")
def oracle_keys():
    """One real client key set (seeded), built by the oracle."""
    from oracle import oracle as O
    import synth
    return O.keygen(synth.key_randomness(KEY_SEED))
