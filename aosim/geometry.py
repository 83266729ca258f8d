"""Pupil geometry of a Shack-Hartmann single-conjugate AO system.

Seeded-input side of the test and benchmark harness: it builds the masks and
coordinates that both the HIP path and the oracle take as *inputs*.  It holds
none of the real-time controller's arithmetic.

Valid-subaperture rule: a subaperture is active when its centre lies inside
the annulus ``obscuration * R <= rho <= R`` with ``R = n_sub / 2`` pitches.
At 80 x 80 subapertures and a 0.25 D central obscuration this gives exactly
the 4708 active subapertures the paper reports for its ELT configuration
(Section 3.1), and it is equivalent there to a >= 50 % illumination rule.

Valid-actuator rule: actuators sit on a Fried grid (the corners of the
subaperture grid, ``n_sub + 1`` per side) and are active within a radius of
``(n_sub + 1) / 2`` pitches of the pupil centre, with no central hole.  For
the paper's 81 x 81 DM this gives 5169, one short of the 5170 it prints
(Section 3.1); the paper does not state its rule.
"""
from __future__ import annotations

import numpy as np


def subaperture_mask(n_sub: int, obscuration: float) -> np.ndarray:
    """uint8 ``[n_sub, n_sub]`` row-major (y outer, x inner); 1 = active.

    Centres are compared in units of half a pitch, so the squared radius is
    an exact integer and the outer edge is tested exactly.
    """
    if n_sub < 1:
        raise ValueError("n_sub must be >= 1")
    if not (0.0 <= obscuration < 1.0):
        raise ValueError("obscuration must be in [0, 1)")
    c = 2 * np.arange(n_sub, dtype=np.int64) + 1 - n_sub  # 2 * centre, in pitches
    r2 = c[None, :] ** 2 + c[:, None] ** 2                # (2 rho)^2
    outer = n_sub * n_sub                                 # (2 R)^2
    inner = (obscuration * n_sub) ** 2
    return ((r2 <= outer) & (r2 >= inner)).astype(np.uint8)


def actuator_mask(n_sub: int) -> np.ndarray:
    """bool ``[n_sub+1, n_sub+1]``: Fried-geometry actuators inside the DM radius."""
    n_act = n_sub + 1
    c = 2 * np.arange(n_act, dtype=np.int64) - n_sub     # 2 * position, in pitches
    r2 = c[None, :] ** 2 + c[:, None] ** 2
    return r2 <= n_act * n_act


def valid_subaperture_cells(mask: np.ndarray) -> np.ndarray:
    """int64 ``[n_valid, 2]`` of (sy, sx), enumerated row-major."""
    sy, sx = np.nonzero(np.asarray(mask) != 0)
    return np.stack([sy, sx], axis=1).astype(np.int64)


def subaperture_boxes(mask: np.ndarray, pitch: float) -> np.ndarray:
    """float64 ``[n_valid, 4]`` = (x0, x1, y0, y1) in metres, pupil centre at 0."""
    n_sub = mask.shape[0]
    cells = valid_subaperture_cells(mask)
    x0 = (cells[:, 1] - n_sub / 2.0) * pitch
    y0 = (cells[:, 0] - n_sub / 2.0) * pitch
    return np.stack([x0, x0 + pitch, y0, y0 + pitch], axis=1)


def actuator_positions(n_sub: int, pitch: float) -> np.ndarray:
    """float64 ``[n_act_valid, 2]`` = (x, y) in metres of the active actuators, row-major."""
    am = actuator_mask(n_sub)
    jy, ix = np.nonzero(am)
    x = (ix - n_sub / 2.0) * pitch
    y = (jy - n_sub / 2.0) * pitch
    return np.stack([x, y], axis=1)
