import functools
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built HIP library")
    config.addinivalue_line("markers", "slow: large workload (tens of seconds on the CPU)")


@functools.lru_cache(maxsize=None)
def cube(n, E=1e5, nu=0.4, seed=999, n_contacts=0):
    import synth

    return synth.cube_system(n, E, nu, seed=seed, n_contacts=n_contacts)


@functools.lru_cache(maxsize=None)
def small_cube():
    import synth

    return synth.config_small()


@functools.lru_cache(maxsize=None)
def large_cube(E=1e6):
    import synth

    return synth.config_large(E=E)


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle

    oracle.lib()
    return oracle
