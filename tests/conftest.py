import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI on the device)")
    config.addinivalue_line("markers", "slow: long CPU test")
    import oracle
    import synth
    synth.build()
    oracle.build()


@pytest.fixture(scope="session")
def c1_graph():
    """Small directed R-MAT graph: scale 16, edge factor 16, seed 1."""
    import synth
    return synth.rmat_csr(16, 16, seed=synth.SEED_GRAPH)
