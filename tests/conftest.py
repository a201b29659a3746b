"""Shared pytest configuration: markers, import path and the oracle build."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU-side oracle runs")


@pytest.fixture(scope="session")
def orc():
    """The FP64 CPU oracle (built on first use)."""
    import oracle
    from oracle import build as ob
    if not os.path.exists(oracle.LIB_PATH):
        ob.build()
    oracle.lib()
    return oracle
