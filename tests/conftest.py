import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU oracle cases")


_ORACLE_CACHE = {}


@pytest.fixture(scope="session")
def oracle_problem():
    """Cached oracle problems keyed by (n_sub, level, coarse_level)."""
    import oracle

    def get(n_sub, level, coarse_level=2):
        key = (n_sub, level, coarse_level)
        if key not in _ORACLE_CACHE:
            _ORACLE_CACHE[key] = oracle.Problem(n_sub, level, coarse_level)
        return _ORACLE_CACHE[key]

    return get
