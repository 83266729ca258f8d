"""Shack-Hartmann detector simulator (harness input generator).

Each active subaperture images a pixel-integrated Gaussian spot whose centre
is displaced from the tile centre by the residual slope (pixels).  Photon
counts are Poisson; the detector adds a dark level and read noise and applies
a per-pixel gain ``1 / flat``, so that a calibration multiplying by ``flat``
restores photo-electrons.  Inactive subapertures see dark + read noise only.
"""
from __future__ import annotations

import numpy as np
from scipy.special import ndtr


def pixel_profile(offset: np.ndarray, n_pix: int, sigma: float) -> np.ndarray:
    """float64 ``[len(offset), n_pix]``: fraction of a unit 1-D Gaussian in each pixel.

    The tile spans [0, n_pix) with its centre at n_pix / 2; ``offset`` moves the
    Gaussian centre (pixels).
    """
    edges = np.arange(n_pix + 1, dtype=np.float64)
    mu = n_pix / 2.0 + np.asarray(offset, dtype=np.float64)[:, None]
    cdf = ndtr((edges[None, :] - mu) / sigma)
    return cdf[:, 1:] - cdf[:, :-1]


def spot_expectation(sx: np.ndarray, sy: np.ndarray, n_pix: int, sigma: float,
                     flux: float) -> np.ndarray:
    """Expected photons, float64 ``[n_valid, n_pix, n_pix]`` (row = y, col = x)."""
    px = pixel_profile(sx, n_pix, sigma)
    py = pixel_profile(sy, n_pix, sigma)
    return flux * py[:, :, None] * px[:, None, :]


def calibration_maps(h: int, w: int, rng: np.random.Generator,
                     dark_level: float = 100.0, dark_sigma: float = 2.0,
                     flat_sigma: float = 0.02) -> tuple[np.ndarray, np.ndarray]:
    """(dark, flat) float32 ``[h, w]``: dark ~ N(100, 2^2) ADU, flat ~ N(1, 0.02^2)."""
    dark = (dark_level + dark_sigma * rng.standard_normal((h, w))).astype(np.float32)
    flat = (1.0 + flat_sigma * rng.standard_normal((h, w))).astype(np.float32)
    return dark, flat


def detector_frame(expected: np.ndarray, mask: np.ndarray, n_pix: int,
                   dark: np.ndarray, flat: np.ndarray, read_noise: float,
                   rng_photon: np.random.Generator, rng_read: np.random.Generator) -> np.ndarray:
    """uint16 ``[H, W]`` raw frame: clip(rint(photons / flat + dark + read), 0, 65535)."""
    n_sub = mask.shape[0]
    h = w = n_sub * n_pix
    photons = np.zeros((h, w), dtype=np.float64)
    sy, sx = np.nonzero(mask)
    counts = rng_photon.poisson(expected)
    tiles = photons.reshape(n_sub, n_pix, n_sub, n_pix)
    tiles[sy, :, sx, :] = counts
    sig = photons / flat.astype(np.float64) + dark.astype(np.float64)
    sig += read_noise * rng_read.standard_normal((h, w))
    return np.clip(np.rint(sig), 0, 65535).astype(np.uint16)
