"""Deformable-mirror model and control-matrix construction (harness inputs).

The interaction matrix ``D`` maps actuator commands to Shack-Hartmann slopes
(in pixels); the control matrix ``R`` is its Tikhonov-regularised
least-squares inverse.  ``R`` is an *input* of the real-time controller: the
controller only multiplies it with the slope vector every frame.

Units: a command of 1 raises the mirror phase by 1 rad (at the sensing
wavelength) at the actuator's own position.  The spot displacement of a
subaperture of side ``d`` is ``d <dphi/dx> / pi`` pixels, i.e. a pixel scale
of lambda / (2 d) (Nyquist sampling of the subaperture diffraction core).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import linalg
from scipy.special import erf


def influence_width(pitch: float, coupling: float = 0.3) -> float:
    """Gaussian width w such that exp(-pitch^2 / 2 w^2) == coupling."""
    return pitch / math.sqrt(2.0 * math.log(1.0 / coupling))


def interaction_matrix(boxes: np.ndarray, acts: np.ndarray, w: float) -> np.ndarray:
    """float64 ``[2 n_valid, n_act]``: x-slope rows first, then y-slope rows.

    Closed form of the mean gradient of ``exp(-r^2 / 2 w^2)`` over each box,
    scaled by ``d / pi`` to pixels.
    """
    x0, x1, y0, y1 = (boxes[:, i][:, None] for i in range(4))
    xa = acts[:, 0][None, :]
    ya = acts[:, 1][None, :]
    d = boxes[0, 1] - boxes[0, 0]
    s2w = math.sqrt(2.0) * w
    g = lambda u: np.exp(-(u * u) / (2.0 * w * w))
    # integral of the Gaussian over an interval, times 1
    gi = lambda a, b, c: w * math.sqrt(math.pi / 2.0) * (erf((b - c) / s2w) - erf((a - c) / s2w))
    dx = (g(x1 - xa) - g(x0 - xa)) * gi(y0, y1, ya)
    dy = (g(y1 - ya) - g(y0 - ya)) * gi(x0, x1, xa)
    scale = 1.0 / (math.pi * d)   # (d / pi) * (1 / d^2)
    return np.concatenate([dx, dy], axis=0) * scale


def tikhonov_control_matrix(D: np.ndarray, alpha: float = 1e-3) -> np.ndarray:
    """float64 ``[n_act, n_slopes]`` = (D^T D + a I)^-1 D^T, a = alpha * trace(D^T D) / n_act."""
    DtD = D.T @ D
    a = alpha * np.trace(DtD) / DtD.shape[0]
    c = linalg.cho_factor(DtD + a * np.eye(DtD.shape[0]), lower=False, check_finite=False)
    return linalg.cho_solve(c, D.T, check_finite=False)


def tikhonov_alpha_abs(D: np.ndarray, alpha: float = 1e-3) -> float:
    """The absolute regulariser a used by :func:`tikhonov_control_matrix`."""
    return float(alpha * np.sum(D * D) / D.shape[1])
