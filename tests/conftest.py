import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long test (a CPU test, or a GPU test at the full workload size)")


_CACHE = {}


def operator(surface="sphere", n=2048, seed=0, leaf=32, eta=1.0, eps_aca=1e-6, eps_comp=1e-6):
    """Seeded operator shared by the tests of one session (built once per parameter set)."""
    from paper_2405_15573_amd import builder, inputs
    key = (surface, n, seed, leaf, eta, eps_aca, eps_comp)
    if key not in _CACHE:
        cloud = inputs.make_cloud(surface, n, seed=seed)
        op = builder.build_operator(cloud, leaf=leaf, eta=eta, eps_aca=eps_aca, eps_comp=eps_comp)
        _CACHE[key] = (cloud, op)
    return _CACHE[key]


@pytest.fixture(scope="session")
def small_op():
    """The N=2048 sphere operator (leaf 32, eta 1, eps 1e-6, seed 0)."""
    return operator()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
