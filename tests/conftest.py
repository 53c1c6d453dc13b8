import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


_CONFIG = None


def pytest_configure(config):
    global _CONFIG
    _CONFIG = config
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: several seconds of CPU work")


def visible(msg: str) -> None:
    """Print past pytest's output capture: progress lines of fixtures that
    take minutes (the problem generation), so that a run stays visibly alive."""
    cm = _CONFIG.pluginmanager.getplugin("capturemanager") if _CONFIG is not None else None
    if cm is None:
        print(msg, flush=True)
        return
    with cm.global_and_fixture_disabled():
        print(msg, flush=True)


_CACHE = {}


def cached(key, fn):
    if key not in _CACHE:
        _CACHE[key] = fn()
    return _CACHE[key]


@pytest.fixture(scope="session")
def hydrogen_small():
    """Hydrogen on 4^3 cells of degree 4 (n ~ 4k), enriched."""
    from synth import configs
    return cached("h4", lambda: configs.hydrogen(nc=4, length=20.0, p=4, r_c=6.0))


@pytest.fixture(scope="session")
def hydrogen_cfg1():
    """The 8^3-cell hydrogen workload (n = 29,793)."""
    from synth import configs
    return cached("h8", lambda: configs.config1())


@pytest.fixture(scope="session")
def si_small():
    """Small Si cluster: 5 atoms, 26 Bohr cube, 8^3 cells (n ~ 33k, n_e = 45)."""
    from synth import configs
    return cached("si5", lambda: configs.si_cluster(n_atoms=5, length=26.0, nc=8, p=4, r_c=8.0,
                                                    seed=3))


@pytest.fixture(scope="session")
def tiny_enriched():
    """Brute-force sized problem: 2^3 cells of degree 2, one atom, 2 enrichments (n ~ 30)."""
    from synth import configs
    return cached("tiny", lambda: configs.hydrogen(nc=2, length=8.0, p=2, r_c=3.0))


def rng(seed=0):
    return np.random.default_rng(seed)


@pytest.fixture(scope="session")
def hydrogen_classical():
    """Hydrogen on 4^3 cells of degree 4 with no enrichment (n_e = 0)."""
    from synth import configs
    return cached("h4c", lambda: configs.hydrogen(nc=4, length=20.0, p=4, enrich=False))


@pytest.fixture(scope="session")
def si_dense():
    """10-atom Si cluster in a 32 Bohr cube on 8^3 cells (n ~ 30k, n_e = 90):
    the central cells meet every atom's support, up to 90 enrichment
    functions per cell (more than one 64-row group of the coupling kernels)."""
    from synth import configs
    return cached("si10", lambda: configs.si_cluster(n_atoms=10, length=32.0, nc=8, p=4,
                                                     r_c=8.0, seed=4))
