"""Frame-time statistics in the paper's terms (Section 3).

Latency is the time from the frame being available to the last DM command
being computed; without a camera it is the frame computation time.  Jitter is
the variation of latency: the RMS jitter is its standard deviation, the
peak-to-peak jitter its range, and the paper also quotes the largest change
between consecutive frames.
"""
from __future__ import annotations

import numpy as np


def frame_stats(t_us: np.ndarray, skip: int = 0) -> dict:
    """Statistics of a per-frame time series in microseconds, after dropping ``skip`` frames."""
    t = np.asarray(t_us, dtype=np.float64)[skip:]
    if t.size == 0:
        raise ValueError("empty series")
    d = np.abs(np.diff(t)) if t.size > 1 else np.zeros(1)
    return {
        "n": int(t.size),
        "mean_us": float(t.mean()),
        "p50_us": float(np.percentile(t, 50)),
        "p99_us": float(np.percentile(t, 99)),
        "min_us": float(t.min()),
        "max_us": float(t.max()),
        "rms_jitter_us": float(t.std()),
        "p2p_jitter_us": float(t.max() - t.min()),
        "max_consecutive_delta_us": float(d.max()),
        "rate_hz": float(1e6 / t.mean()),
    }


def ticks_to_us(ticks: np.ndarray, khz: int) -> np.ndarray:
    """Device wall-clock ticks (rate in kHz) to microseconds."""
    return np.asarray(ticks, dtype=np.float64) * (1000.0 / float(khz))
