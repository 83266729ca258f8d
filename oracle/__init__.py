"""FP64 CPU oracle of the AO real-time-control hot path.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke entry point
and the benchmark's CPU-baseline leg, never by the product library.

Parity status: every function is pinned by tests against closed forms,
exact rational arithmetic or brute force (see ``tests/test_oracle_pins.py``);
none is "parity unpinned".
"""
from .rtc_oracle import (FrameOracle, calibrate, centroids, integrate, reconstruct,  # noqa: F401
                         rtc_frame, rtc_frame_multi, sensor_slopes, slope_vector, subaperture_tiles,
                         threshold_excess, valid_subapertures)
