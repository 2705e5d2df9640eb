"""Error counting against a per-codeword loop; Wilson interval against
scipy's binomtest(...).proportion_ci(method="wilson")."""
import numpy as np
import pytest
from scipy import stats as sst

from inputs import rand
from oracle import stats


def test_count_errors_loop():
    u = rand.bits(1, (50, 37))
    h = u.copy()
    r = rand.rng(2)
    for b in range(50):
        n = int(r.integers(0, 4))
        for i in r.choice(37, n, replace=False):
            h[b, i] ^= 1
    bins = r.integers(0, 3, 50)
    got = stats.count_errors(u, h, bins, 3)
    for k in range(3):
        be = sum(int((u[b] != h[b]).sum()) for b in range(50) if bins[b] == k)
        bl = sum(int((u[b] != h[b]).any()) for b in range(50) if bins[b] == k)
        assert got[k].tolist() == [be, bl, int((bins == k).sum())]


@pytest.mark.parametrize("k,n", [(0, 100), (3, 1000), (50, 100), (999, 1000), (7, 7)])
def test_wilson_vs_scipy(k, n):
    ci = sst.binomtest(k, n).proportion_ci(confidence_level=0.95, method="wilson")
    lo, hi = stats.wilson(k, n)
    assert abs(lo - ci.low) < 1e-6 and abs(hi - ci.high) < 1e-6
