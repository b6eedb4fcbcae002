import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

U = 2.0 ** -53  # FP64 unit round-off (Sec. III)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running (full-size workloads)")


def rand_mw(rng, k, n, emin=-20, emax=20, normalised=True):
    """Random k-word numbers: a leading word with a random exponent and each
    lower word at most 2^-54 of the one above (normalised), or up to 2^-50
    of it (overlapping, as quasi values may be)."""
    w0 = rng.uniform(-1.0, 1.0, n) * 2.0 ** rng.integers(emin, emax, n).astype(np.float64)
    planes = [w0]
    shrink = 2.0 ** -54 if normalised else 2.0 ** -50
    for _ in range(1, k):
        planes.append(planes[-1] * rng.uniform(-1.0, 1.0, n) * shrink)
    return np.ascontiguousarray(np.stack(planes))


@pytest.fixture
def rng():
    return np.random.default_rng(12345)
