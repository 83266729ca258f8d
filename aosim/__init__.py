"""Seeded synthetic AO inputs: pupil geometry, DM/interaction/control matrices,
von Karman frozen-flow turbulence and a Shack-Hartmann detector simulator.

Shared by the parity tests and the benchmark as an *input source* only.  It
contains none of the real-time controller's per-frame arithmetic
(calibration, centroiding, reconstruction, integration).
"""
from .scenario import CONFIGS, ELT, TINY, ScaoConfig, Scenario, rng_for  # noqa: F401
