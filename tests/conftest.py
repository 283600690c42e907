import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


KEY_SEED = 0x5EED0001


@pytest.fixture(scope="session")
def oracle_keys():
    """One real client key set (seeded), built by the oracle."""
    from oracle import oracle as O
    import synth
    return O.keygen(synth.key_randomness(KEY_SEED))
