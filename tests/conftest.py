import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: oracle runs that take tens of seconds")


_GRIDS = {}


def oracle_grid(g, smooth=True, k=100.0, scalar_atan2=False):
    """Session cache of oracle grids (building one at g6 takes ~30 s, a
    minute with the C library's atan2)."""
    from oracle import grid
    key = (g, smooth, k, scalar_atan2)
    if key not in _GRIDS:
        _GRIDS[key] = grid.Grid(g, smooth=smooth, k=k, scalar_atan2=scalar_atan2)
    return _GRIDS[key]


@pytest.fixture(scope="session")
def ogrid():
    return oracle_grid
