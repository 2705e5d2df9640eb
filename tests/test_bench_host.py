"""Host-side logic of bench.py (no GPU): the one-GPU guard, the Eb/N0 read
off a BLER curve, and the guard that drops counter traffic taken on other
kernel sources."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_ebn0_at_bler_interpolates_in_log_bler():
    # 1e-1 at 1 dB and 1e-3 at 2 dB: 1e-2 is halfway in log10 BLER
    assert bench.ebn0_at_bler([0.0, 1.0, 2.0], [1.0, 1e-1, 1e-3]) == pytest.approx(1.5)
    # the first crossing only (a noisy curve may cross again)
    assert bench.ebn0_at_bler([0.0, 1.0, 2.0, 3.0], [1.0, 1e-3, 0.5, 1e-3]) == pytest.approx(2 / 3)
    # a point with no block errors past the target: that point
    assert bench.ebn0_at_bler([0.0, 1.0], [0.5, 0.0]) == 1.0
    # never below the target
    assert bench.ebn0_at_bler([0.0, 1.0], [1.0, 0.5]) is None


def test_traffic_is_dropped_for_other_sources():
    for entry in (bench.LAYERED_TRAFFIC, bench.FLOOD_SPA_TRAFFIC):
        stale = dict(entry, sha256_16="0" * 16)
        assert bench._traffic(stale) is None
        assert bench._traffic(dict(entry, bytes=None)) is None
