"""Reduced-precision control-matrix storage: encoder and decoder (oracle side).

TEST INFRASTRUCTURE.  Shares no code with the HIP library's encoder.

Section 2.3.4 of the paper stores the control matrix as IEEE binary16 to halve
the bytes the bandwidth-bound reconstruction reads, and converts each value
to 32-bit before the multiply-accumulate.  The same idea is extended here to
bfloat16 and to OCP FP8 E4M3 (e4m3fn), each with one float32 scale per
matrix row:

  * scale: s_r = 2^e_r with e_r the smallest integer such that
    max_j |R_rj| / 2^e_r <= 2^E (E = 15 for binary16, 0 for bfloat16, 8 for
    E4M3), clamped to [-126, 127]; e_r = 0 for an all-zero row;
  * code: R_rj / s_r (exact, s_r is a power of two) rounded to the nearest
    value of the format, ties to the even significand, the sign kept on zero;
  * value: decode(code) * s_r; the multiply-accumulate is float32.

Formats (sign, exponent bits, fraction bits, bias, largest finite):
  binary16 1-5-10, 15, 65504;  bfloat16 1-8-7, 127, (2 - 2^-7) 2^127;
  E4M3    1-4-3, 7, 448 (no infinities; S.1111.111 is NaN and never produced).
"""
from __future__ import annotations

import numpy as np

FORMATS = {
    # name: (exp_bits, frac_bits, bias, E, code dtype)
    "f16": (5, 10, 15, 15, np.uint16),
    "bf16": (8, 7, 127, 0, np.uint16),
    "fp8e4m3": (4, 3, 7, 8, np.uint8),
}


def row_scale_exponents(R: np.ndarray, fmt: str) -> np.ndarray:
    """e_r per row: smallest integer with max|R_r| / 2^e_r <= 2^E, clamped to [-126, 127]."""
    E = FORMATS[fmt][3]
    m = np.max(np.abs(np.asarray(R, dtype=np.float64)), axis=1)
    mant, ex = np.frexp(m)                       # m = mant * 2^ex, mant in [0.5, 1)
    ceil_log2 = np.where(mant == 0.5, ex - 1, ex)
    e = np.where(m == 0.0, 0, ceil_log2 - E)
    return np.clip(e, -126, 127).astype(np.int64)


def round_to_format(y: np.ndarray, fmt: str) -> np.ndarray:
    """Nearest value of the format (ties to even significand), float64, |y| within range."""
    ebits, fbits, bias, _, _ = FORMATS[fmt]
    y = np.asarray(y, dtype=np.float64)
    a = np.abs(y)
    _, ex = np.frexp(a)                          # a in [2^(ex-1), 2^ex)
    exp_unb = np.maximum(ex - 1, 1 - bias)       # subnormals share the lowest binade's spacing
    quantum = np.ldexp(1.0, exp_unb - fbits)     # spacing of representable values near a
    r = np.rint(a / quantum) * quantum           # rint: round half to even
    r = np.where(a == 0.0, 0.0, r)
    return np.copysign(r, y)


def _value_to_code(v: np.ndarray, fmt: str) -> np.ndarray:
    ebits, fbits, bias, _, cdt = FORMATS[fmt]
    nbits = 1 + ebits + fbits
    sign = np.signbit(v).astype(np.int64)
    a = np.abs(v)
    _, ex = np.frexp(a)
    normal = (a >= np.ldexp(1.0, 1 - bias))
    e_field = np.where(normal, ex - 1 + bias, 0)
    frac = np.where(normal, np.ldexp(a, -(ex - 1) + fbits) - (1 << fbits),
                    np.ldexp(a, bias - 1 + fbits))
    frac = np.where(a == 0.0, 0, frac).astype(np.int64)
    code = (sign << (nbits - 1)) | (e_field.astype(np.int64) << fbits) | frac
    return code.astype(cdt)


def encode(R: np.ndarray, fmt: str):
    """(codes [n_rows, n_cols], scales float32 [n_rows]) of a float32 matrix."""
    R = np.asarray(R, dtype=np.float32).astype(np.float64)
    e = row_scale_exponents(R, fmt)
    y = np.ldexp(R, -e[:, None])                 # exact
    v = round_to_format(y, fmt)
    return _value_to_code(v, fmt), np.ldexp(1.0, e).astype(np.float32)


def decode_codes(codes: np.ndarray, fmt: str) -> np.ndarray:
    """float64 value of each code, from the format's definition."""
    ebits, fbits, bias, _, _ = FORMATS[fmt]
    nbits = 1 + ebits + fbits
    c = np.asarray(codes).astype(np.int64)
    sign = np.where((c >> (nbits - 1)) & 1, -1.0, 1.0)
    e_field = (c >> fbits) & ((1 << ebits) - 1)
    frac = (c & ((1 << fbits) - 1)).astype(np.float64)
    normal = np.ldexp(1.0 + frac / (1 << fbits), e_field - bias)
    sub = np.ldexp(frac / (1 << fbits), 1 - bias)
    return sign * np.where(e_field == 0, sub, normal)


def dequantize(codes: np.ndarray, scales: np.ndarray, fmt: str) -> np.ndarray:
    """The matrix the reduced-precision reconstruction multiplies, float64."""
    return decode_codes(codes, fmt) * np.asarray(scales, dtype=np.float64)[:, None]


def unit_roundoff(fmt: str) -> float:
    """Relative rounding bound for normal values: 2^-(fraction bits + 1)."""
    return 2.0 ** -(FORMATS[fmt][1] + 1)
