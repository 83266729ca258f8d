"""Reduced-precision control-matrix storage: oracle encoder pins and byte-exact
agreement of the library's host encoder (no GPU needed)."""
import numpy as np
import pytest
import torch

from oracle import quant
from paper_1805_07254_amd import rtc

FMTS = ["f16", "bf16", "fp8e4m3"]
LIB_ID = {"f16": rtc.RTC_CM_F16, "bf16": rtc.RTC_CM_BF16, "fp8e4m3": rtc.RTC_CM_FP8E4M3}


def _lib_round(y32: np.ndarray, fmt: str) -> np.ndarray:
    """The format's rounding of float32 values by numpy / torch conversion routines."""
    if fmt == "f16":
        return y32.astype(np.float16).astype(np.float64)
    t = torch.from_numpy(y32)
    dt = torch.bfloat16 if fmt == "bf16" else torch.float8_e4m3fn
    return t.to(dt).to(torch.float64).numpy()


def _in_range_values(fmt, rng, n=20000):
    E = quant.FORMATS[fmt][3]
    # magnitudes spanning normals and subnormals of the format, below 2^E
    lo = {"f16": -26, "bf16": -136, "fp8e4m3": -11}[fmt]
    ex = rng.uniform(lo, E, n)
    y = (rng.choice([-1.0, 1.0], n) * 2.0 ** ex).astype(np.float32)
    return y


@pytest.mark.parametrize("fmt", FMTS)
def test_rounding_matches_library_conversions(fmt):
    y = _in_range_values(fmt, np.random.default_rng(1))
    ours = quant.round_to_format(y.astype(np.float64), fmt)
    assert np.array_equal(ours, _lib_round(y, fmt))


@pytest.mark.parametrize("fmt", FMTS)
def test_rounding_matches_brute_force_nearest_with_ties_to_even(fmt):
    nb = 1 + quant.FORMATS[fmt][0] + quant.FORMATS[fmt][1]
    codes = np.arange(1 << nb)
    vals = quant.decode_codes(codes, fmt)
    ok = np.isfinite(vals) & (codes >> (nb - 1) == 0)
    if fmt == "fp8e4m3":
        ok &= (codes & 0x7F) != 0x7F                   # S.1111.111 is NaN in e4m3fn
    else:
        ok &= ((codes >> quant.FORMATS[fmt][1]) & ((1 << quant.FORMATS[fmt][0]) - 1)) != (1 << quant.FORMATS[fmt][0]) - 1
    pos_codes, pos_vals = codes[ok], vals[ok]
    order = np.argsort(pos_vals)
    pos_codes, pos_vals = pos_codes[order], pos_vals[order]
    rng = np.random.default_rng(2)
    y = np.abs(_in_range_values(fmt, rng, 3000)).astype(np.float64)
    # add exact midpoints between neighbours (ties) and grid points
    k = min(200, len(pos_vals) - 1)
    mids = (pos_vals[1:k + 1] + pos_vals[:k]) / 2
    y = np.concatenate([y, mids, pos_vals[:50]])
    got = quant.round_to_format(y, fmt)
    for yi, gi in zip(y, got):
        k = np.searchsorted(pos_vals, yi)
        cands = [j for j in (k - 1, k) if 0 <= j < len(pos_vals)]
        d = [abs(pos_vals[j] - yi) for j in cands]
        best = [cands[i] for i in range(len(cands)) if d[i] == min(d)]
        if len(best) == 2:                                  # tie: even significand (even code)
            best = [j for j in best if pos_codes[j] % 2 == 0]
        assert gi == pos_vals[best[0]], (fmt, yi, gi)


@pytest.mark.parametrize("fmt", FMTS)
def test_row_scale_is_smallest_power_of_two(fmt):
    rng = np.random.default_rng(3)
    R = (rng.standard_normal((40, 17)) * 10.0 ** rng.uniform(-30, 30, (40, 1))).astype(np.float32)
    R[5] = 0.0
    R[6, 3] = 2.0 ** 20                                    # exact power of two maximum
    E = quant.FORMATS[fmt][3]
    e = quant.row_scale_exponents(R, fmt)
    for r in range(R.shape[0]):
        m = float(np.max(np.abs(R[r].astype(np.float64))))
        if m == 0.0:
            assert e[r] == 0
            continue
        want = next(k for k in range(-400, 400) if m / 2.0 ** k <= 2.0 ** E)
        assert e[r] == min(127, max(-126, want))


@pytest.mark.parametrize("fmt", FMTS)
def test_quantisation_error_bound(fmt):
    rng = np.random.default_rng(4)
    R = rng.standard_normal((64, 300)).astype(np.float32)
    codes, scales = quant.encode(R, fmt)
    Rq = quant.dequantize(codes, scales, fmt)
    u = quant.unit_roundoff(fmt)
    bias, fbits = quant.FORMATS[fmt][2], quant.FORMATS[fmt][1]
    sub = np.ldexp(1.0, 1 - bias - fbits - 1) * scales[:, None].astype(np.float64)   # half the subnormal step
    assert np.all(np.abs(Rq - R) <= np.maximum(u * np.abs(R), sub))
    assert np.all(np.abs(Rq) <= np.abs(R).max(axis=1, keepdims=True) * (1 + u))


def _hard_matrix(rng, fmt):
    """Rows with wide dynamic range, exact ties, zeros and signed zeros."""
    R = rng.standard_normal((32, 257)).astype(np.float32)
    R[:8] *= (10.0 ** rng.uniform(-6, 0, (8, 257))).astype(np.float32)    # subnormal codes
    R[8] = 0.0
    R[9] = -0.0
    R[9, 0] = 1.0
    # exact ties: a grid point plus half the spacing of the format at the row's scale
    fbits = quant.FORMATS[fmt][1]
    R[10] = 1.0
    R[10, 1:100] = np.float32(1.0) + np.float32(2.0 ** -(fbits + 1)) * (np.arange(1, 100) % 2).astype(np.float32)
    R[11] = (rng.standard_normal(257) * 1e30).astype(np.float32)
    R[12] = (rng.standard_normal(257) * 1e-30).astype(np.float32)
    R[13] = np.float32(3.4e38) * np.sign(rng.standard_normal(257)).astype(np.float32)
    return R


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_library_encoder_is_byte_identical_to_oracle(fmt, seed):
    rng = np.random.default_rng(10 + seed)
    R = _hard_matrix(rng, fmt) if seed == 0 else (rng.standard_normal((50, 333)) *
                                                   10.0 ** rng.uniform(-5, 5, (50, 1))).astype(np.float32)
    oc, osc = quant.encode(R, fmt)
    lc, lsc = rtc.rtc_encode_cmat(LIB_ID[fmt], R)
    if seed == 0:   # the tie row really holds ties: half of its scaled entries sit on midpoints
        y = np.ldexp(R[10].astype(np.float64), -int(np.log2(osc[10])))
        assert np.sum(quant.round_to_format(y, fmt) != y) >= 49
    assert lc.dtype == oc.dtype
    assert np.array_equal(lsc, osc)
    assert np.array_equal(lc, oc)


def test_encoder_rejects_bad_arguments():
    with pytest.raises(rtc.RtcError) as ei:
        rtc.rtc_encode_cmat(rtc.RTC_CM_F32, np.ones((2, 2), np.float32))
    assert ei.value.status == rtc.RTC_E_ARG
    bad = np.ones((2, 2), np.float32)
    bad[1, 1] = np.nan
    with pytest.raises(rtc.RtcError) as ei:
        rtc.rtc_encode_cmat(rtc.RTC_CM_BF16, bad)
    assert ei.value.status == rtc.RTC_E_NONFINITE


def _library_view(codes: np.ndarray, fmt: str) -> np.ndarray:
    """float64 value of each bit pattern as numpy / torch read the same bits."""
    if fmt == "f16":
        return codes.astype(np.uint16).view(np.float16).astype(np.float64)
    if fmt == "bf16":
        return torch.from_numpy(codes.astype(np.uint16).view(np.int16)).view(torch.bfloat16).to(torch.float64).numpy()
    return torch.from_numpy(codes.astype(np.uint8)).view(torch.float8_e4m3fn).to(torch.float64).numpy()


@pytest.mark.parametrize("fmt", FMTS)
def test_every_code_has_the_library_bit_layout(fmt):
    # decode_codes and _value_to_code against the bits numpy and torch assign:
    # every finite pattern decodes to the library's value (signed zeros
    # included) and encodes back to the same pattern
    nb = 1 + quant.FORMATS[fmt][0] + quant.FORMATS[fmt][1]
    codes = np.arange(1 << nb, dtype=np.int64)
    lib = _library_view(codes, fmt)
    finite = np.isfinite(lib)
    assert finite.sum() == {"f16": 63488, "bf16": 65280, "fp8e4m3": 254}[fmt]
    ours = quant.decode_codes(codes, fmt)
    assert np.array_equal(ours[finite], lib[finite])
    assert np.array_equal(np.signbit(ours[finite]), np.signbit(lib[finite]))
    back = quant._value_to_code(lib[finite], fmt).astype(np.int64)
    assert np.array_equal(back, codes[finite])
