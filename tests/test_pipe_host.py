"""Host logic of pixel-stream processing that needs no GPU: the subaperture
allocation (linearly decreasing counts per worker, Section 3.2) and argument
checks of the pixel-stream entry points."""
import ctypes
import math

import numpy as np
import pytest

from paper_1805_07254_amd import rtc


def _targets(n, P, ratio):
    w = np.array([1.0] if P == 1 else [ratio + (1.0 - ratio) * b / (P - 1) for b in range(P)])
    return n * w / w.sum()


@pytest.mark.parametrize("n,P,ratio", [(3972, 255, 1.0), (3972, 255, 8.0), (3972, 255, 1000.0), (80, 7, 3.0),
                                       (80, 255, 1.0), (80, 255, 5.0), (0, 10, 2.0), (1, 1, 1.0), (97, 1, 40.0),
                                       (12345, 1024, 2.5)])
def test_allocation_is_the_linear_rule_rounded(n, P, ratio):
    c = rtc.rtc_pipe_allocation(n, P, ratio).astype(np.int64)
    assert c.shape == (P,) and c.min() >= 0 and c.sum() == n
    x = _targets(n, P, ratio)
    assert np.all(np.abs(c - x) < 1.0)                 # floor or ceil of each worker's linear share
    assert np.all(np.diff(c) <= 0)                     # earlier pixels, more subapertures
    if P > 2:
        assert np.abs(np.diff(c, 2)).max() <= 2        # linear up to rounding


@pytest.mark.parametrize("n,P", [(3972, 255), (80, 7), (5, 9), (1024, 1024)])
def test_equal_allocation_is_floor_or_ceil_with_extras_first(n, P):
    q, r = divmod(n, P)
    assert rtc.rtc_pipe_allocation(n, P, 1.0).tolist() == [q + 1] * r + [q] * (P - r)


def test_allocation_first_to_last_ratio():
    c = rtc.rtc_pipe_allocation(100000, 100, 10.0)
    assert abs(c[0] / c[-1] - 10.0) < 0.1
    # shares fall by the same amount per worker: (ratio - 1) / (P - 1) of the last one's
    step = np.diff(c.astype(np.float64))
    assert np.allclose(step, step.mean(), atol=1.0)


@pytest.mark.parametrize("n,P,ratio", [(-1, 4, 1.0), (10, 0, 1.0), (10, 4, 0.5), (10, 4, math.nan),
                                       (10, 4, 1001.0)])
def test_allocation_rejects_bad_arguments(n, P, ratio):
    with pytest.raises(rtc.RtcError) as e:
        rtc.rtc_pipe_allocation(n, P, ratio)
    assert e.value.status == rtc.RTC_E_ARG


def test_pipe_entry_points_reject_null_context():
    lib = rtc.load_library()
    cfg = rtc.rtc_pipe_config(n_workers=0, full_frame=0, alloc_ratio=1.0, frame_period_us=1000.0,
                              readout_us=1000.0, rows_per_packet=2, wait_limit_us=0, tail_rows=0,
                              reserved=0)
    assert lib.rtc_pipe_setup(None, ctypes.byref(cfg)) == rtc.RTC_E_ARG
    assert lib.rtc_pipe_info(None, None, None, None, None, None, None) == rtc.RTC_E_ARG
    assert lib.rtc_pipe_run(None, 1, None, 0, None, None, None, None, None, None, None) == rtc.RTC_E_ARG
    assert lib.rtc_pipe_allocation(4, 2, 1.0, None) == rtc.RTC_E_ARG
    assert ctypes.sizeof(rtc.rtc_pipe_config) == 48
