"""Seeded constructed inputs shared by the oracle pins and the GPU parity tests."""
from __future__ import annotations

import numpy as np


def near_tie_pixels(seed: int = 7, n_candidates: int = 400000, T: float | None = None,
                    flat_range=(0.9, 1.1)):
    """Pixels whose calibrated value lies within ~1e-11 relative of the threshold.

    For float32 T (random per pixel, or the given fixed value) and random float32
    flat, raw = ceil(T / flat) and dark = raw - T / flat rounded to float32, kept
    where 2^-13 <= dark < 2^-12 (inside the domain where raw - dark is exact in
    float64).  Returns (raw uint16, dark f32, flat f32, T f32) 1-D arrays.
    """
    rng = np.random.default_rng(seed)
    if T is None:
        Tv = rng.uniform(1000, 60000, n_candidates).astype(np.float32)
    else:
        Tv = np.full(n_candidates, T, dtype=np.float32)
    flat = rng.uniform(flat_range[0], flat_range[1], n_candidates).astype(np.float32)
    dstar = Tv.astype(np.float64) / flat.astype(np.float64)
    raw = np.ceil(dstar)
    dark = raw - dstar
    ok = (dark >= 2.0 ** -13) & (dark < 2.0 ** -12) & (raw <= 65535)
    return (raw[ok].astype(np.uint16), dark[ok].astype(np.float32), flat[ok], Tv[ok])


def pixel_integrated_gaussian(n: int, offset: float, sigma: float) -> np.ndarray:
    """Fraction of a unit 1-D Gaussian centred at n/2 + offset in each of n pixels."""
    from scipy.special import ndtr
    edges = np.arange(n + 1, dtype=np.float64)
    cdf = ndtr((edges - (n / 2.0 + offset)) / sigma)
    return cdf[1:] - cdf[:-1]


def out_of_domain_tie_pixels(T: float = 3.0):
    """Pixels whose calibrated value ties or nearly ties T with darks outside
    [2^-13, 2^24) in magnitude, where raw - dark is not exact in float64.

    Exact ties of raw * flat with T (raw a power of two, flat = T / raw exact)
    shifted by tiny darks of both signs (normal and subnormal float32), the
    same with darks of magnitude 2^60 and flats of the opposite sign, and
    zero darks at the exact tie (a tie counts as below).  Returns (raw uint16,
    dark f32, flat f32) 1-D arrays for the float32 threshold T.
    """
    raw, dark, flat = [], [], []
    T32 = np.float32(T)
    for k in range(0, 16):
        r = 2 ** k
        f = np.float32(T32 / np.float32(r))
        if np.float64(r) * np.float64(f) != np.float64(T32):
            continue
        for dk in (-149, -140, -126, -100, -60, -40, -31):
            if np.log2(r) - (dk - 23 if dk > -127 else -149) < 53:
                continue                        # raw - dark would be exact in float64
            for sgn in (1.0, -1.0):
                raw.append(r)
                dark.append(np.float32(sgn * 2.0 ** dk))
                flat.append(f)
        raw.append(r)
        dark.append(np.float32(0.0))
        flat.append(f)
    for r in (1, 5, 77, 65535):
        for sgn in (1.0, -1.0):
            d = np.float32(sgn * 2.0 ** 60)
            f = np.float32(-sgn * np.float64(T32) * 2.0 ** -60)
            raw.append(r)
            dark.append(d)
            flat.append(f)
    return (np.asarray(raw, dtype=np.uint16), np.asarray(dark, dtype=np.float32),
            np.asarray(flat, dtype=np.float32))
