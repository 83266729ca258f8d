"""Pins of the FP64 oracle against closed forms, exact arithmetic and brute force.

Each test checks the oracle against something other than itself: values the
paper prints, analytic results, exact rational arithmetic or enumeration.
"""
from fractions import Fraction
import math
import os

import numpy as np
import pytest

import oracle
from aosim import dm, geometry
from _cases import near_tie_pixels, out_of_domain_tie_pixels, pixel_integrated_gaussian

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                out[k] = float(v) if "." in v else int(v)
    return out


# ---------------------------------------------------------------- index map
def test_index_map_row_major_enumeration():
    mask = np.array([[0, 1, 1], [1, 0, 0], [0, 0, 1]], dtype=np.uint8)
    cells = oracle.valid_subapertures(mask)
    assert cells.tolist() == [[0, 1], [0, 2], [1, 0], [2, 2]]


def test_paper_elt_geometry_count():
    g = _golden("paper_elt_geometry.txt")
    mask = geometry.subaperture_mask(g["n_sub"], g["obscuration"])
    cells = oracle.valid_subapertures(mask)
    assert len(cells) == g["active_subapertures"]
    assert 2 * len(cells) == g["slopes"]
    # The radius rule gives one actuator fewer than the paper prints for 81 x 81.
    assert geometry.actuator_mask(g["dm_side"] - 1).sum() == g["actuators"] - 1


@pytest.mark.parametrize("n_sub,obs,nv,nact", [(10, 0.0, 80, 97), (74, 0.28, 3972, 4421),
                                               (16, 0.28, 192, 225)])
def test_config_geometry_counts(n_sub, obs, nv, nact):
    assert len(oracle.valid_subapertures(geometry.subaperture_mask(n_sub, obs))) == nv
    assert geometry.actuator_mask(n_sub).sum() == nact


def test_tile_extraction_brute_force():
    n_sub, n = 5, 3
    mask = geometry.subaperture_mask(n_sub, 0.3)
    img = (np.arange(n_sub * n)[:, None] * 1000 + np.arange(n_sub * n)[None, :]).astype(np.int64)
    cells = oracle.valid_subapertures(mask)
    tiles = oracle.subaperture_tiles(img, cells, n)
    k = 0
    for sy in range(n_sub):
        for sx in range(n_sub):
            if mask[sy, sx]:
                for i in range(n):
                    for j in range(n):
                        assert tiles[k, i, j] == (sy * n + i) * 1000 + sx * n + j
                k += 1
    assert k == len(cells)


# --------------------------------------------------------------- calibration
def test_calibration_dyadic_values_exact():
    raw = np.array([[[103, 104], [100, 104]]], dtype=np.uint16)
    dark = np.array([[[100.25, 100.25], [100.25, 100.0]]], dtype=np.float32)
    flat = np.array([[[1.125, 1.125], [1.125, 0.75]]], dtype=np.float32)
    # x = (raw - dark) * flat: 3.09375, 4.21875, -0.28125, 3.0 (== T: below)
    v, counts = oracle.calibrate(raw, dark, flat, 3.0, "subtract")
    assert v.tolist() == [[[0.09375, 1.21875], [0.0, 0.0]]]
    assert counts.tolist() == [2]
    v, counts = oracle.calibrate(raw, dark, flat, 3.0, "zero")
    assert v.tolist() == [[[3.09375, 4.21875], [0.0, 0.0]]]
    assert counts.tolist() == [2]


def test_calibration_order_dark_then_flat():
    # (raw - dark) * flat differs from raw * flat - dark and from (raw - dark) / flat.
    raw = np.array([[[120]]], dtype=np.uint16)
    dark = np.array([[[100.0]]], dtype=np.float32)
    flat = np.array([[[0.5]]], dtype=np.float32)
    v, _ = oracle.calibrate(raw, dark, flat, 0.0, "zero")
    assert v[0, 0, 0] == 10.0


def test_threshold_near_ties_exact():
    raw, dark, flat, T = near_tie_pixels()
    assert len(raw) > 20
    naive_wrong = 0
    for i in range(len(raw)):
        exact = (Fraction(int(raw[i])) - Fraction(float(dark[i]))) * Fraction(float(flat[i])) \
            - Fraction(float(T[i]))
        above, x, y = oracle.threshold_excess(raw[i:i + 1], dark[i:i + 1], flat[i:i + 1], T[i])
        assert bool(above[0]) == (exact > 0)
        assert y[0] == float(exact)
        naive = (float(raw[i]) - float(dark[i])) * float(flat[i]) - float(T[i])
        naive_wrong += (naive > 0) != (exact > 0)
    assert naive_wrong > 0, "construction no longer produces float64-ambiguous ties"


def test_threshold_random_pixels_match_exact_decisions():
    rng = np.random.default_rng(11)
    raw = rng.integers(90, 130, size=(4, 6, 6)).astype(np.uint16)
    dark = (100 + 2 * rng.standard_normal((4, 6, 6))).astype(np.float32)
    flat = (1 + 0.02 * rng.standard_normal((4, 6, 6))).astype(np.float32)
    T = np.float32(3.0)
    above, x, y = oracle.threshold_excess(raw, dark, flat, T)
    for idx in np.ndindex(raw.shape):
        ex = (Fraction(int(raw[idx])) - Fraction(float(dark[idx]))) * Fraction(float(flat[idx])) \
            - Fraction(float(T))
        assert bool(above[idx]) == (ex > 0)
        assert abs(y[idx] - float(ex)) <= 4 * 2.0 ** -53 * (abs(x[idx]) + float(T))


def test_threshold_exact_for_darks_outside_the_fast_domain():
    # tiny (down to subnormal) and 2^60 darks, where raw - dark is not exact in
    # float64: the oracle's decisions equal exact rational arithmetic, and plain
    # float64 gets a good share of these ties wrong
    raw, dark, flat = out_of_domain_tie_pixels(3.0)
    above, x, y = oracle.threshold_excess(raw, dark, flat, 3.0)
    naive_wrong = 0
    for i in range(len(raw)):
        ex = (Fraction(int(raw[i])) - Fraction(float(dark[i]))) * Fraction(float(flat[i])) - 3
        assert bool(above[i]) == (ex > 0), i
        assert y[i] == float(ex)
        naive = (float(raw[i]) - float(dark[i])) * float(flat[i]) - 3.0
        naive_wrong += (naive > 0) != (ex > 0)
    assert naive_wrong > 20 and above.any() and not above.all()


def test_mode_none_keeps_every_calibrated_value():
    # x = (raw - dark) * flat: 3.09375, 4.21875, -0.28125, 3.0; nothing is clipped
    raw = np.array([[[103, 104], [100, 104]]], dtype=np.uint16)
    dark = np.array([[[100.25, 100.25], [100.25, 100.0]]], dtype=np.float32)
    flat = np.array([[[1.125, 1.125], [1.125, 0.75]]], dtype=np.float32)
    v, counts = oracle.calibrate(raw, dark, flat, 3.0, "none")
    assert v.tolist() == [[[3.09375, 4.21875], [-0.28125, 3.0]]]
    assert counts.tolist() == [2]                    # still the pixels above T
    cx, cy = oracle.centroids(v, counts)
    S = Fraction(309375 + 421875 - 28125 + 300000, 100000)
    assert cx[0] == float((Fraction(-1, 2) * (Fraction(309375, 100000) - Fraction(28125, 100000))
                           + Fraction(1, 2) * (Fraction(421875, 100000) + 3)) / S)
    assert cy[0] == float((Fraction(-1, 2) * (Fraction(309375 + 421875, 100000))
                           + Fraction(1, 2) * (Fraction(-28125, 100000) + 3)) / S)


def test_mode_none_equals_mode_zero_when_every_pixel_is_above():
    rng = np.random.default_rng(5)
    raw = rng.integers(150, 400, size=(6, 8, 8)).astype(np.uint16)
    dark = (100 + 2 * rng.standard_normal((6, 8, 8))).astype(np.float32)
    flat = (1 + 0.02 * rng.standard_normal((6, 8, 8))).astype(np.float32)
    v0, c0 = oracle.calibrate(raw, dark, flat, 3.0, "zero")
    vn, cn = oracle.calibrate(raw, dark, flat, 3.0, "none")
    assert np.all(c0 == 64) and np.array_equal(c0, cn) and np.array_equal(v0, vn)


def test_mode_none_slopes_do_not_depend_on_the_threshold():
    rng = np.random.default_rng(6)
    raw = rng.integers(90, 200, size=(5, 6, 6)).astype(np.uint16)
    dark = np.full((5, 6, 6), 100.0, np.float32)
    flat = np.ones((5, 6, 6), np.float32)
    out = [oracle.calibrate(raw, dark, flat, T, "none") for T in (0.0, 3.0, 50.0)]
    for v, c in out[1:]:
        assert np.array_equal(v, out[0][0])
    assert out[0][1].sum() > out[1][1].sum() > out[2][1].sum()


def test_mode_none_nonpositive_sum_gives_zero_centroid():
    # every pixel below the dark: S < 0; S == 0 with mixed signs; both centroid 0
    raw = np.array([[[90, 95], [98, 99]], [[110, 90], [100, 100]]], dtype=np.uint16)
    dark = np.full((2, 2, 2), 100.0, np.float32)
    flat = np.ones((2, 2, 2), np.float32)
    v, counts = oracle.calibrate(raw, dark, flat, 0.0, "none")
    assert v.sum(axis=(1, 2)).tolist() == [-18.0, 0.0]
    cx, cy = oracle.centroids(v, counts)
    assert cx.tolist() == [0.0, 0.0] and cy.tolist() == [0.0, 0.0]


def test_threshold_must_be_nonnegative():
    with pytest.raises(ValueError):
        oracle.calibrate(np.zeros((1, 1, 1), np.uint16), np.zeros((1, 1, 1), np.float32),
                         np.ones((1, 1, 1), np.float32), -1.0)


# ------------------------------------------------------------ centre of gravity
@pytest.mark.parametrize("dx,dy", [(0.1, -0.25), (0.5, 0.0), (-1.0, 0.37), (2.2, -1.6)])
def test_cog_of_gaussian_spot_on_wide_window_is_offset(dx, dy):
    # Poisson summation: the pixelisation bias is below exp(-2 pi^2 sigma^2) / pi ~ 1.5e-13 px.
    n, sigma = 64, 1.2
    v = 500.0 * np.outer(pixel_integrated_gaussian(n, dy, sigma), pixel_integrated_gaussian(n, dx, sigma))
    cx, cy = oracle.centroids(v[None], np.array([n * n]))
    assert abs(cx[0] - dx) < 1e-12 and abs(cy[0] - dy) < 1e-12


@pytest.mark.parametrize("n", [8, 10])
@pytest.mark.parametrize("dx,dy", [(0.1, 0.25), (0.5, -1.0), (1.0, 0.1)])
def test_cog_on_detector_window_matches_separable_closed_form(n, dx, dy):
    sigma = 1.2
    px, py = pixel_integrated_gaussian(n, dx, sigma), pixel_integrated_gaussian(n, dy, sigma)
    pos = np.arange(n) + 0.5 - n / 2.0
    ex, ey = (pos * px).sum() / px.sum(), (pos * py).sum() / py.sum()
    cx, cy = oracle.centroids((500.0 * np.outer(py, px))[None], np.array([n * n]))
    assert abs(cx[0] - ex) < 1e-13 and abs(cy[0] - ey) < 1e-13
    # truncation pulls the estimate towards the centre
    assert abs(cx[0]) < abs(dx) and abs(cy[0]) < abs(dy)


def test_uniform_illumination_gives_exactly_zero_slopes():
    raw = np.full((3, 10, 10), 150, dtype=np.uint16)
    dark = np.full((3, 10, 10), 100.0, dtype=np.float32)
    flat = np.ones((3, 10, 10), dtype=np.float32)
    v, counts = oracle.calibrate(raw, dark, flat, 3.0)
    cx, cy = oracle.centroids(v, counts)
    assert counts.tolist() == [100] * 3
    assert np.all(cx == 0.0) and np.all(cy == 0.0)


def test_integer_tiles_give_correctly_rounded_quotients():
    rng = np.random.default_rng(3)
    v = rng.integers(0, 200, size=(16, 8, 8)).astype(np.float64)
    counts = (v > 0).reshape(16, -1).sum(1)
    cx, cy = oracle.centroids(v, counts)
    for k in range(16):
        S = sum(Fraction(int(t)) for t in v[k].ravel())
        Sx = sum(Fraction(2 * j - 7, 2) * int(v[k, i, j]) for i in range(8) for j in range(8))
        Sy = sum(Fraction(2 * i - 7, 2) * int(v[k, i, j]) for i in range(8) for j in range(8))
        assert cx[k] == float(Sx / S) and cy[k] == float(Sy / S)


def test_empty_subaperture_gives_minus_reference():
    raw = np.full((2, 4, 4), 100, dtype=np.uint16)
    raw[1, 1, 2] = 140
    dark = np.full((2, 4, 4), 100.0, dtype=np.float32)
    flat = np.ones((2, 4, 4), dtype=np.float32)
    v, counts = oracle.calibrate(raw, dark, flat, 3.0)
    assert counts.tolist() == [0, 1]
    cx, cy = oracle.centroids(v, counts)
    ref = np.array([0.5, -0.25, 0.125, 1.0], dtype=np.float32)
    s = oracle.slope_vector(cx, cy, ref)
    # tile 0: nothing above -> centroid 0; tile 1: single pixel at (row 1, col 2)
    assert s.tolist() == [-0.5, 0.5 + 0.25, -0.125, -0.5 - 1.0]


def test_slope_layout_x_block_then_y_block():
    # Section 2.1: subaperture i puts its x gradient at s_i and its y gradient at s_{n/2+i}.
    nv, n = 5, 6
    v = np.ones((nv, n, n))
    col = np.array([1, 2, 3, 5, 8, 13], dtype=np.float64)   # asymmetric in x
    row = np.array([2, 7, 9, 9, 7, 2], dtype=np.float64)    # mirror-symmetric in y
    v[3] = np.outer(row, col)
    cx, cy = oracle.centroids(v, np.full(nv, n * n))
    s = oracle.slope_vector(cx, cy)
    expect_x = float(sum(Fraction(2 * j - 5, 2) * int(c) for j, c in enumerate(col)) / int(col.sum()))
    assert s[3] == expect_x and s[nv + 3] == 0.0
    assert np.all(np.delete(s, 3) == 0.0)


# --------------------------------------------------------------------- MVM
def test_mvm_brute_force_exact_sum():
    rng = np.random.default_rng(5)
    for n_act, n_s in [(3, 8), (6, 6), (8, 16)]:
        R = rng.standard_normal((n_act, n_s)).astype(np.float32)
        s = rng.standard_normal(n_s)
        a = oracle.reconstruct(R, s)
        for r in range(n_act):
            exact = sum(Fraction(float(R[r, j])) * Fraction(float(s[j])) for j in range(n_s))
            bound = n_s * 2.0 ** -53 * sum(abs(float(R[r, j]) * s[j]) for j in range(n_s))
            assert abs(a[r] - float(exact)) <= bound


def test_mvm_orientation_rows_are_actuators():
    R = np.array([[1, 2, 3, 4]], dtype=np.float32)    # 1 actuator, 4 slopes
    assert oracle.reconstruct(R, np.array([1.0, 0.0, 0.0, 1.0])).tolist() == [5.0]


# --------------------------------------------------------------- integrator
def test_integrator_constant_input_closed_form():
    a = np.array([3.0, -2.0, 7.0])
    c = np.array([1.0, 1.0, -4.0])
    c0 = c.copy()
    for k in range(1, 21):
        c = oracle.integrate(c, a, gain=0.5, leak=1.0)
        assert c.tolist() == (c0 + k * 0.5 * a).tolist()


def test_leaky_integrator_closed_form():
    lam, g = float(np.float32(0.99)), float(np.float32(0.4))
    a = np.array([0.7, -1.3])
    c0 = np.array([2.0, -0.5])
    c = c0.copy()
    for k in range(1, 51):
        c = oracle.integrate(c, a, gain=0.4, leak=0.99)
        ref = lam ** k * c0 + g * a * (1 - lam ** k) / (1 - lam)
        assert np.allclose(c, ref, rtol=1e-12, atol=0)


def test_integrator_clamp():
    c = oracle.integrate(np.zeros(3), np.array([10.0, -10.0, 0.1]), 1.0, 1.0, -1.0, 1.0)
    assert c.tolist() == [1.0, -1.0, float(np.float32(1.0)) * 0.1]


def test_closed_loop_modal_convergence_with_tikhonov_matrix():
    # Static aberration, geometric slopes s_k = s* - D c_{k-1}: along the SVD modes of D,
    # c_k = (1 - (1 - g s^2/(s^2+a))^k) u / s exactly (no noise, no pixels).
    mask = geometry.subaperture_mask(10, 0.0)
    pitch = 0.2
    D = dm.interaction_matrix(geometry.subaperture_boxes(mask, pitch),
                              geometry.actuator_positions(10, pitch), dm.influence_width(pitch))
    R = dm.tikhonov_control_matrix(D, 1e-3)
    alpha = dm.tikhonov_alpha_abs(D, 1e-3)
    U, sig, Vt = np.linalg.svd(D, full_matrices=False)
    rng = np.random.default_rng(2)
    s_star = D @ rng.standard_normal(D.shape[1]) + 0.1 * rng.standard_normal(D.shape[0])
    g = float(np.float32(0.4))
    u = U.T @ s_star
    c = np.zeros(D.shape[1])
    for k in range(1, 31):
        c = oracle.integrate(c, oracle.reconstruct(R, s_star - D @ c), gain=0.4)
        z = (1 - (1 - g * sig ** 2 / (sig ** 2 + alpha)) ** k) * u / sig
        assert np.allclose(Vt @ c, z, rtol=0, atol=1e-10 * np.abs(u / sig).max())


# ------------------------------------------------------------- whole frame
def test_frame_composes_steps_on_full_frame():
    rng = np.random.default_rng(9)
    n_sub, n = 6, 4
    mask = geometry.subaperture_mask(n_sub, 0.2)
    H = n_sub * n
    frame = rng.integers(95, 160, size=(H, H)).astype(np.uint16)
    dark = (100 + rng.standard_normal((H, H))).astype(np.float32)
    flat = (1 + 0.02 * rng.standard_normal((H, H))).astype(np.float32)
    nv = int(mask.sum())
    R = rng.standard_normal((7, 2 * nv)).astype(np.float32)
    c_prev = rng.standard_normal(7)
    out = oracle.rtc_frame(frame, mask, n, dark, flat, 3.0, R, c_prev, 0.4)
    cells = oracle.valid_subapertures(mask)
    for k, (sy, sx) in enumerate(cells):
        sl = np.s_[sy * n:(sy + 1) * n, sx * n:(sx + 1) * n]
        v, cnt = oracle.calibrate(frame[sl][None], dark[sl][None], flat[sl][None], 3.0)
        cx, cy = oracle.centroids(v, cnt)
        assert out["counts"][k] == cnt[0]
        assert out["slopes"][k] == cx[0] and out["slopes"][nv + k] == cy[0]
    assert np.array_equal(out["recon"], R.astype(np.float64) @ out["slopes"])
    fo = oracle.FrameOracle(mask, n, dark, flat, 3.0, R, 0.4)
    out2 = fo(frame, c_prev)
    for key in out:
        assert np.array_equal(out[key], out2[key])
