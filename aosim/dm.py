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
    scaled by ``d / pi`` to pixels.  Each entry is a product of a factor of
    (box x edges, actuator x) and a factor of (box y edges, actuator y); the
    factors are evaluated once per distinct pair and gathered.
    """
    d = boxes[0, 1] - boxes[0, 0]
    s2w = math.sqrt(2.0) * w
    g = lambda u: np.exp(-(u * u) / (2.0 * w * w))
    # integral of the Gaussian over an interval, times 1
    gi = lambda a, b, c: w * math.sqrt(math.pi / 2.0) * (erf((b - c) / s2w) - erf((a - c) / s2w))

    def tables(lo, hi, pos):
        ul, il = np.unique(lo, return_inverse=True)
        up, ip = np.unique(pos, return_inverse=True)
        lo_u = ul[:, None]
        hi_u = (ul + (hi[0] - lo[0]))[:, None] if np.all(hi - lo == hi[0] - lo[0]) else None
        if hi_u is None:                                    # unequal boxes: one row per box
            lo_u, hi_u, il = lo[:, None], hi[:, None], np.arange(len(lo))
        p = up[None, :]
        return g(hi_u - p) - g(lo_u - p), gi(lo_u, hi_u, p), il, ip

    x0, x1, y0, y1 = (boxes[:, i] for i in range(4))
    gx, ix_int, bx, ax = tables(x0, x1, acts[:, 0])
    gy, iy_int, by, ay = tables(y0, y1, acts[:, 1])
    dx = gx[bx[:, None], ax[None, :]] * iy_int[by[:, None], ay[None, :]]
    dy = gy[by[:, None], ay[None, :]] * ix_int[bx[:, None], ax[None, :]]
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
