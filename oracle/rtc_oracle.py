"""FP64 CPU oracle of the per-frame adaptive-optics real-time-control path.

TEST INFRASTRUCTURE.  Only the test suite, the smoke entry point and the
benchmark's CPU-baseline leg may import this module.  It shares no code,
tables or constants with the HIP implementation and never calls it.

What one frame computes (Jenkins, Basden & Myers 2018, Section 2.1 and the
Figure 3 caption; Section 2.2 for per-subaperture processing):

  (a) pixel calibration of every active subaperture: background (dark)
      subtraction, flat-field application, threshold application, in that
      order;
  (b) a centre-of-gravity centroid per subaperture, written into the slope
      vector with all x gradients first and then all y gradients
      (subaperture i -> s_i and s_{n/2 + i});
  (c) wavefront reconstruction: control matrix times slope vector
      (Section 1.1.1: N slope measurements, M actuators);
  (d) a gain applied to the reconstruction to form the actuator commands,
      taken as an integrator c_k = leak * c_{k-1} + gain * a_k.

Readings where the paper is silent (each also listed in the design notes):
  * threshold: the calibrated value x = (raw - dark) * flat is compared with
    the threshold T by the sign of the *exact* real number x - T, strictly
    (x == T counts as below).  Mode "subtract": v = x - T above, else 0.
    Mode "zero": v = x above, else 0.  Mode "none": v = x for every pixel
    (no threshold applied; counts still report the pixels above T).  T >= 0.
    Any finite dark and flat are accepted.
  * flat field multiplies (the map holds inverse pixel gains).
  * centroid coordinates are in pixels from the tile centre, (n-1)/2,
    +x along increasing column, +y along increasing row; a subaperture whose
    weighted sum is not positive has centroid 0 (with a threshold: no pixel
    above it).  Optional reference slopes are subtracted.
  * active subapertures are enumerated row-major over the mask; subaperture
    k covers rows [sy n, sy n + n) and columns [sx n, sx n + n).
  * the control matrix R is [n_act][n_slopes] so that a = R s.

Everything is evaluated in float64 from the exact float32 / uint16 inputs.
The threshold decision falls back to exact rational arithmetic
(fractions.Fraction) for pixels whose float64 value of x - T lies within a
rigorous error band of zero, so decisions and counts are exact.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

MODES = ("subtract", "zero", "none")

# |fl64(fl64(fl64(raw - dark) * flat) - T) - (x - T)| <= 3 * 2^-53 * (|x| + |T|);
# anything within this (much wider) band is re-decided exactly.
_TIE_BAND = 1e-12


def valid_subapertures(mask: np.ndarray) -> np.ndarray:
    """(sy, sx) of every active subaperture, row-major; int64 ``[n_valid, 2]``."""
    mask = np.asarray(mask)
    cells = []
    for sy in range(mask.shape[0]):
        for sx in range(mask.shape[1]):
            if mask[sy, sx] != 0:
                cells.append((sy, sx))
    return np.asarray(cells, dtype=np.int64).reshape(-1, 2)


def subaperture_tiles(image: np.ndarray, cells: np.ndarray, n_pix: int) -> np.ndarray:
    """Pixel tiles ``[n_valid, n_pix, n_pix]`` (row = y, col = x) of a full-frame array."""
    out = np.empty((len(cells), n_pix, n_pix), dtype=image.dtype)
    for k, (sy, sx) in enumerate(cells):
        out[k] = image[sy * n_pix:(sy + 1) * n_pix, sx * n_pix:(sx + 1) * n_pix]
    return out


def _exact_excess(raw: int, dark: float, flat: float, T: float) -> Fraction:
    """(raw - dark) * flat - T as an exact rational."""
    return (Fraction(int(raw)) - Fraction(float(dark))) * Fraction(float(flat)) - Fraction(float(T))


def threshold_excess(raw: np.ndarray, dark: np.ndarray, flat: np.ndarray, T: float):
    """Calibrated value and its excess over T, with exact threshold decisions.

    Returns ``(above, x, y)``: ``above`` is the exact decision x - T > 0,
    ``x`` = (raw - dark) * flat and ``y`` = x - T in float64 (the correctly
    rounded exact value wherever the fast float64 evaluation was ambiguous).
    """
    T64 = float(np.float32(T))
    x = (raw.astype(np.float64) - dark.astype(np.float64)) * flat.astype(np.float64)
    y = x - T64
    above = y > 0.0
    near = np.abs(y) <= _TIE_BAND * (np.abs(x) + abs(T64))
    for idx in zip(*np.nonzero(near)):
        ex = _exact_excess(raw[idx], dark[idx], flat[idx], T64)
        above[idx] = ex > 0
        y[idx] = float(ex)
        x[idx] = float(ex + Fraction(T64))
    return above, x, y


def calibrate(raw: np.ndarray, dark: np.ndarray, flat: np.ndarray, T: float, mode: str = "subtract"):
    """Background, flat field, threshold (Figure 3 (a)); returns ``(v, counts)``.

    ``raw`` uint16, ``dark``/``flat`` float32 tiles ``[n_valid, n, n]``.
    ``v`` float64 tiles, ``counts`` int64 ``[n_valid]`` = pixels above T.
    """
    if mode not in MODES:
        raise ValueError(f"mode must be one of {MODES}")
    if not (float(T) >= 0.0):
        raise ValueError("threshold must be >= 0")
    above, x, y = threshold_excess(raw, dark, flat, T)
    if mode == "none":
        v = x.copy()
    else:
        v = np.where(above, y if mode == "subtract" else x, 0.0)
    counts = above.reshape(above.shape[0], -1).sum(axis=1).astype(np.int64)
    return v, counts


def centroids(v: np.ndarray, counts: np.ndarray):
    """Centre of gravity of each tile (Figure 3 (b)); returns ``(cx, cy)`` float64.

    ``cx = sum(xc * v) / sum(v)`` with ``xc = col - (n - 1) / 2`` (and rows
    for y); 0 where ``sum(v)`` is not positive.  With a threshold applied
    every v is >= 0 and positive exactly above the threshold, so that is the
    subapertures with no pixel above it (``counts`` 0).
    """
    n = v.shape[-1]
    xc = np.arange(n, dtype=np.float64) - (n - 1) / 2.0
    S = v.sum(axis=(1, 2))
    Sx = (v * xc[None, None, :]).sum(axis=(1, 2))
    Sy = (v * xc[None, :, None]).sum(axis=(1, 2))
    has = S > 0.0
    safe = np.where(has, S, 1.0)
    return np.where(has, Sx / safe, 0.0), np.where(has, Sy / safe, 0.0)


def slope_vector(cx: np.ndarray, cy: np.ndarray, ref: np.ndarray | None = None) -> np.ndarray:
    """x gradients of all subapertures, then all y gradients, minus reference slopes."""
    s = np.concatenate([cx, cy]).astype(np.float64)
    if ref is not None:
        s = s - np.asarray(ref, dtype=np.float32).astype(np.float64)
    return s


def reconstruct(R: np.ndarray, s: np.ndarray) -> np.ndarray:
    """a = R s (Figure 3 (c)); R ``[n_act, n_slopes]``, promoted to float64."""
    return np.asarray(R).astype(np.float64) @ np.asarray(s, dtype=np.float64)


def integrate(c_prev: np.ndarray, a: np.ndarray, gain: float, leak: float = 1.0,
              cmd_min: float = -np.inf, cmd_max: float = np.inf) -> np.ndarray:
    """c = leak * c_prev + gain * a, clamped to [cmd_min, cmd_max] (Figure 3 (d))."""
    g = float(np.float32(gain))
    lam = float(np.float32(leak))
    c = lam * np.asarray(c_prev, dtype=np.float64) + g * np.asarray(a, dtype=np.float64)
    return np.clip(c, float(np.float32(cmd_min)), float(np.float32(cmd_max)))


def rtc_frame(frame: np.ndarray, mask: np.ndarray, n_pix: int, dark: np.ndarray, flat: np.ndarray,
              T: float, R: np.ndarray, c_prev: np.ndarray, gain: float, leak: float = 1.0,
              mode: str = "subtract", ref: np.ndarray | None = None,
              cmd_min: float = -np.inf, cmd_max: float = np.inf) -> dict:
    """One frame of the hot path on a full uint16 frame and full-frame dark/flat maps."""
    cells = valid_subapertures(mask)
    raw_t = subaperture_tiles(frame, cells, n_pix)
    dark_t = subaperture_tiles(dark, cells, n_pix)
    flat_t = subaperture_tiles(flat, cells, n_pix)
    v, counts = calibrate(raw_t, dark_t, flat_t, T, mode)
    cx, cy = centroids(v, counts)
    s = slope_vector(cx, cy, ref)
    a = reconstruct(R, s)
    c = integrate(c_prev, a, gain, leak, cmd_min, cmd_max)
    return {"counts": counts, "slopes": s, "recon": a, "cmd": c}


def sensor_slopes(frame: np.ndarray, mask: np.ndarray, n_pix: int, dark: np.ndarray, flat: np.ndarray,
                  T: float, mode: str = "subtract"):
    """Steps (a)-(b) of one wavefront sensor: (slopes x block then y block, counts)."""
    cells = valid_subapertures(mask)
    v, counts = calibrate(subaperture_tiles(frame, cells, n_pix), subaperture_tiles(dark, cells, n_pix),
                          subaperture_tiles(flat, cells, n_pix), T, mode)
    cx, cy = centroids(v, counts)
    return slope_vector(cx, cy), counts


def rtc_frame_multi(frames, sensors, darks, flats, thresholds, R: np.ndarray, c_prev: np.ndarray, gain: float,
                    leak: float = 1.0, mode: str = "subtract", ref: np.ndarray | None = None,
                    cmd_min: float = -np.inf, cmd_max: float = np.inf) -> dict:
    """One frame of several wavefront sensors reconstructed by one matrix.

    The paper runs one sensor and names multi-sensor systems as its outlook
    (Section 3.4.1) without fixing a layout; here each sensor's slope vector
    (x block then y block, as in Figure 3 (b)) is concatenated in sensor
    order, reference slopes are subtracted from the concatenation, and R is
    [n_act][total slopes].  ``sensors`` is a sequence of (mask, n_pix);
    frames, darks, flats and thresholds follow the same order.
    """
    parts, counts = [], []
    for frame, (mask, n_pix), dark, flat, T in zip(frames, sensors, darks, flats, thresholds):
        s_w, c_w = sensor_slopes(frame, mask, n_pix, dark, flat, T, mode)
        parts.append(s_w)
        counts.append(c_w)
    s = np.concatenate(parts)
    if ref is not None:
        s = s - np.asarray(ref, dtype=np.float32).astype(np.float64)
    a = reconstruct(R, s)
    c = integrate(c_prev, a, gain, leak, cmd_min, cmd_max)
    return {"counts": np.concatenate(counts), "slopes": s, "recon": a, "cmd": c}


class FrameOracle:
    """The same frame with the tile extraction and matrix promotion done once.

    Used for timing the oracle over many frames; the arithmetic per frame is
    exactly that of :func:`rtc_frame`.
    """

    def __init__(self, mask, n_pix, dark, flat, T, R, gain, leak=1.0, mode="subtract",
                 ref=None, cmd_min=-np.inf, cmd_max=np.inf):
        self.cells = valid_subapertures(mask)
        self.n_pix = n_pix
        self.dark_t = subaperture_tiles(dark, self.cells, n_pix)
        self.flat_t = subaperture_tiles(flat, self.cells, n_pix)
        self.T, self.mode, self.ref = T, mode, ref
        self.R64 = np.asarray(R).astype(np.float64)
        self.gain, self.leak, self.cmd_min, self.cmd_max = gain, leak, cmd_min, cmd_max

    def __call__(self, frame: np.ndarray, c_prev: np.ndarray) -> dict:
        raw_t = subaperture_tiles(frame, self.cells, self.n_pix)
        v, counts = calibrate(raw_t, self.dark_t, self.flat_t, self.T, self.mode)
        cx, cy = centroids(v, counts)
        s = slope_vector(cx, cy, self.ref)
        a = self.R64 @ s
        c = integrate(c_prev, a, self.gain, self.leak, self.cmd_min, self.cmd_max)
        return {"counts": counts, "slopes": s, "recon": a, "cmd": c}
