"""Frozen-flow von Karman phase screens and geometric Shack-Hartmann slopes.

Harness input generator only.  Screens are periodic FFT screens (one complex
draw gives two independent real screens); the phase is in radians at the
sensing wavelength (500 nm).  Frozen flow moves the screen by an integer
number of samples per frame, so no interpolation is needed.
"""
from __future__ import annotations

import numpy as np


def von_karman_psd(f: np.ndarray, r0: float, L0: float) -> np.ndarray:
    """Phase power spectral density [rad^2 m^2] at spatial frequency f [cycles/m]."""
    return 0.023 * r0 ** (-5.0 / 3.0) * (f * f + 1.0 / (L0 * L0)) ** (-11.0 / 6.0)


def _psd_grid(n: int, delta: float, r0: float, L0: float) -> tuple[np.ndarray, float]:
    df = 1.0 / (n * delta)
    fx = np.fft.fftfreq(n, d=delta)
    f2 = fx[None, :] ** 2 + fx[:, None] ** 2
    psd = von_karman_psd(np.sqrt(f2), r0, L0)
    psd[0, 0] = 0.0
    return psd, df


def phase_screen_pair(n: int, delta: float, r0: float, L0: float,
                      rng: np.random.Generator) -> tuple[np.ndarray, np.ndarray]:
    """Two independent periodic screens, float64 ``[n, n]`` (rows = y, cols = x)."""
    psd, df = _psd_grid(n, delta, r0, L0)
    amp = np.sqrt(psd) * df
    c = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) * amp
    scr = np.fft.ifft2(c) * (n * n)
    return scr.real.copy(), scr.imag.copy()


def expected_structure_function(n: int, delta: float, r0: float, L0: float,
                                lags: np.ndarray) -> np.ndarray:
    """E[(phi(x + r) - phi(x))^2] along x for the discrete screen construction above."""
    psd, df = _psd_grid(n, delta, r0, L0)
    fx = np.fft.fftfreq(n, d=delta)
    out = []
    for r in np.atleast_1d(lags):
        out.append(2.0 * np.sum(psd * df * df * (1.0 - np.cos(2 * np.pi * fx[None, :] * r * delta))))
    return np.asarray(out)


def geometric_slopes(window: np.ndarray, mask: np.ndarray, m: int) -> np.ndarray:
    """Mean-gradient slopes in pixels, float64 ``[2 n_valid]`` (x block, then y block).

    ``window`` is the phase over the pupil, sampled on ``n_sub * m + 1`` points
    per side (subaperture edges fall on samples); ``m`` samples per pitch.
    The slope of a subaperture is the trapezoid mean, along the edge, of the
    phase difference across it, divided by pi (see :mod:`aosim.dm` units).
    """
    n_sub = mask.shape[0]
    npts = n_sub * m + 1
    if window.shape != (npts, npts):
        raise ValueError("window must be (n_sub*m+1) square")
    return edge_slopes(window[:, ::m], window[::m, :], mask, m)


def edge_slopes(cols: np.ndarray, rows: np.ndarray, mask: np.ndarray, m: int) -> np.ndarray:
    """:func:`geometric_slopes` from the window's subaperture-edge samples only:
    ``cols`` = window[:, ::m] ``[npts, n_sub + 1]``, ``rows`` = window[::m, :]
    ``[n_sub + 1, npts]``."""
    w = np.ones(m + 1)
    w[0] = w[-1] = 0.5
    sy, sx = np.nonzero(mask)
    # edge-difference profiles: dxp[y, i] = phi(y, (i+1) m) - phi(y, i m)
    dxp = cols[:, 1:] - cols[:, :-1]          # [npts, n_sub]
    dyp = rows[1:, :] - rows[:-1, :]          # [n_sub, npts]
    # trapezoid mean along the edge for every subaperture
    idx = np.arange(m + 1)
    ys = sy[:, None] * m + idx[None, :]       # [nv, m+1]
    xs = sx[:, None] * m + idx[None, :]
    gx = (dxp[ys, sx[:, None]] * w).sum(axis=1) / m
    gy = (dyp[sy[:, None], xs] * w).sum(axis=1) / m
    return np.concatenate([gx, gy]) / np.pi
