import numpy as np
import pytest

from paper_1805_07254_amd.stats import frame_stats, ticks_to_us


def test_frame_stats_hand_computed():
    t = np.array([10.0, 12.0, 11.0, 15.0, 12.0])
    s = frame_stats(t)
    assert s["n"] == 5
    assert s["mean_us"] == 12.0
    assert s["p50_us"] == 12.0
    assert s["min_us"] == 10.0 and s["max_us"] == 15.0
    assert s["p2p_jitter_us"] == 5.0
    assert s["max_consecutive_delta_us"] == 4.0
    assert s["rms_jitter_us"] == pytest.approx(np.sqrt((4 + 0 + 1 + 9 + 0) / 5))
    assert s["rate_hz"] == pytest.approx(1e6 / 12.0)


def test_frame_stats_skip_startup_and_spike():
    t = np.full(1000, 20.0)
    t[0] = 500.0          # start-up frame
    t[700] = 80.0         # one outlier
    s_all, s_skip = frame_stats(t), frame_stats(t, skip=100)
    assert s_all["max_us"] == 500.0 and s_skip["max_us"] == 80.0
    assert s_skip["max_consecutive_delta_us"] == 60.0
    assert s_skip["p50_us"] == 20.0 and s_skip["p99_us"] == 20.0
    assert s_skip["rms_jitter_us"] == pytest.approx(60.0 * np.sqrt(1 / 900 - 1 / 900 ** 2))


def test_ticks_to_us():
    assert ticks_to_us(np.array([100, 250]), 100000).tolist() == [1.0, 2.5]
