import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


def _ensure_cpu_libs():
    from paper_1711_06571_amd import datagen
    import oracle
    if not os.path.exists(datagen._LIB):
        datagen.build_lib()
    if not os.path.exists(oracle._LIB):
        oracle.build_lib()


_ensure_cpu_libs()


@pytest.fixture(scope="session")
def rng():
    return np.random.default_rng(12345)


def upper_index(i, j):
    """Position of (i, j), i <= j, in the 21-entry upper triangle."""
    if i > j:
        i, j = j, i
    return i * 6 - i * (i - 1) // 2 + (j - i)


def full_from_upper(u):
    """(21, n) -> (n, 6, 6)."""
    n = u.shape[1]
    P = np.zeros((n, 6, 6), dtype=u.dtype)
    for i in range(6):
        for j in range(i, 6):
            P[:, i, j] = u[upper_index(i, j)]
            P[:, j, i] = u[upper_index(i, j)]
    return P


def upper_from_full(P):
    """(n, 6, 6) -> (21, n)."""
    n = P.shape[0]
    u = np.zeros((21, n), dtype=P.dtype)
    for i in range(6):
        for j in range(i, 6):
            u[upper_index(i, j)] = P[:, i, j]
    return u
