import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle as O
    O.build()
    return O


@pytest.fixture(scope="session")
def pairs_in_cutoff_ok():
    """Checks a GPU system's count of pairs within r_c against the float64
    oracle in the same state.  The float64 form decides r < r_c as the oracle
    does, so the counts are equal.  The mixed form decides it on a float32
    r^2 (one rounded difference per axis, then the rounded sum: a relative
    error below 1e-6 of r^2), so a pair whose float64 distance lies within
    1e-6 of r_c, relative, may count either way: the count must lie between
    the oracle's counts at r_c (1 -+ 1e-6)."""
    def check(o, rc, n_gpu, n_ref, prec):
        if prec == "fp64":
            return n_gpu == n_ref
        assert len(o.pairset(rc)) == n_ref
        lo, hi = len(o.pairset(rc * (1.0 - 1e-6))), len(o.pairset(rc * (1.0 + 1e-6)))
        if not lo <= n_gpu <= hi:
            print("pairs in cutoff", n_gpu, "outside", (lo, hi))
        return lo <= n_gpu <= hi
    return check
