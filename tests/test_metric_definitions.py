"""The benchmark's metric definitions against the numbers the paper prints.

Sec. 4, Table 5 gives, per receiver version, the average tracking time per
1 ms epoch per channel and the number of real-time tracking channels it
implies.  bench.realtime_channels must reproduce the printed counts from the
printed times (channels x data seconds / wall seconds)."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _table5():
    rows = []
    with open(os.path.join(ROOT, "tests", "golden", "paper_table5_offline_tracking.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, ns, ch = line.strip().split("|")
            rows.append((name, float(ns), float(ch)))
    return rows


@pytest.mark.parametrize("name,ns,printed", _table5())
def test_realtime_channels_reproduce_table5(name, ns, printed):
    # one channel, one 1 ms epoch of data, processed in `ns` nanoseconds
    got = bench.realtime_channels(1, 1e-3, ns * 1e-9)
    assert round(got, 2) == pytest.approx(printed, abs=1e-9), (name, got)


def test_realtime_channels_scale_with_channels_and_data():
    # 12 channels x 10 s of data in 0.5 s of wall time: 240 real-time channels
    assert bench.realtime_channels(12, 10.0, 0.5) == pytest.approx(240.0)


def test_table5_speedup_matches_text():
    # Sec. 4 states the SIMD version is up to 6.8x faster than the base version
    rows = {r[0]: r[1] for r in _table5()}
    assert rows["base version"] / rows["SIMD"] == pytest.approx(6.8, abs=0.05)
