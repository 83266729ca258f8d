"""Checks of the seeded input generator (geometry, DM model, turbulence, detector)."""
import math

import numpy as np
from scipy import integrate

from aosim import TINY, Scenario, dm, geometry, shwfs, turbulence


def test_interaction_matrix_matches_quadrature():
    pitch = 0.2
    w = dm.influence_width(pitch, 0.3)
    assert math.isclose(math.exp(-pitch ** 2 / (2 * w * w)), 0.3, rel_tol=1e-14)
    box = np.array([[0.05, 0.25, -0.1, 0.1]])
    act = np.array([[0.1, 0.03], [0.4, -0.2]])
    D = dm.interaction_matrix(box, act, w)
    for j, (xa, ya) in enumerate(act):
        phi = lambda y, x: math.exp(-((x - xa) ** 2 + (y - ya) ** 2) / (2 * w * w))
        dphidx = lambda y, x: -(x - xa) / (w * w) * phi(y, x)
        dphidy = lambda y, x: -(y - ya) / (w * w) * phi(y, x)
        gx = integrate.dblquad(dphidx, 0.05, 0.25, -0.1, 0.1, epsabs=1e-13)[0] / pitch ** 2
        gy = integrate.dblquad(dphidy, 0.05, 0.25, -0.1, 0.1, epsabs=1e-13)[0] / pitch ** 2
        assert abs(D[0, j] - pitch * gx / math.pi) < 1e-8
        assert abs(D[1, j] - pitch * gy / math.pi) < 1e-8


def test_tikhonov_cholesky_matches_svd_filter_factors():
    sc = Scenario(TINY)
    D = sc.interaction
    R = dm.tikhonov_control_matrix(D, 1e-3)
    a = dm.tikhonov_alpha_abs(D, 1e-3)
    U, s, Vt = np.linalg.svd(D, full_matrices=False)
    R_svd = Vt.T @ np.diag(s / (s * s + a)) @ U.T
    assert np.abs(R - R_svd).max() <= 1e-10 * np.abs(R_svd).max()
    assert sc.control_matrix.dtype == np.float32 and sc.control_matrix.shape == (97, 160)


def test_geometric_slopes_of_tilt_and_gradient_scaling():
    # phase = t * x (rad, x in samples): every subaperture sees t * m samples of phase
    # difference across it -> slope t * m / pi px in x, 0 in y.
    mask = geometry.subaperture_mask(4, 0.0)
    m = 5
    n = 4 * m + 1
    t = 0.03
    win = t * np.arange(n)[None, :] * np.ones((n, 1))
    s = turbulence.geometric_slopes(win, mask, m)
    nv = int(mask.sum())
    assert np.allclose(s[:nv], t * m / math.pi, rtol=1e-14) and np.allclose(s[nv:], 0, atol=1e-15)


def test_screen_structure_function_matches_its_spectrum():
    n, delta, r0, L0 = 256, 0.02, 0.15, 25.0
    rng = np.random.default_rng(1)
    lags = np.array([1, 4, 16])
    acc = np.zeros(len(lags))
    reps = 6
    for _ in range(reps):
        a, b = turbulence.phase_screen_pair(n, delta, r0, L0, rng)
        for scr in (a, b):
            acc += [np.mean((np.roll(scr, -L, axis=1) - scr) ** 2) for L in lags]
    emp = acc / (2 * reps)
    theory = turbulence.expected_structure_function(n, delta, r0, L0, lags)
    assert np.all(np.abs(emp / theory - 1) < 0.08), (emp, theory)
    # and the small-lag value follows Kolmogorov 6.88 (r/r0)^(5/3) within the L0/grid deficit
    kol = 6.88 * (lags * delta / r0) ** (5 / 3)
    assert 0.75 < theory[0] / kol[0] < 1.05


def test_detector_frame_statistics_and_seeding():
    sc = Scenario(TINY)
    s = sc.turbulence_slopes(3)
    f1 = sc.frame(3, s)
    f2 = sc.frame(3, s)
    assert f1.dtype == np.uint16 and f1.shape == (80, 80)
    assert np.array_equal(f1, f2)
    assert not np.array_equal(f1, sc.frame(4, s))
    # photo-electrons after calibration ~ flux per subaperture (window truncation < 0.2 %)
    cal = (f1.astype(np.float64) - sc.dark) * sc.flat
    tiles = cal.reshape(10, 8, 10, 8).transpose(0, 2, 1, 3)[sc.mask.astype(bool)]
    assert abs(tiles.sum(axis=(1, 2)).mean() / TINY.flux - 1) < 0.02


def test_spot_expectation_centre_and_flux():
    e = shwfs.spot_expectation(np.array([0.0, 0.5]), np.array([0.0, -0.3]), 10, 1.2, 500.0)
    assert abs(e[0].sum() - 500.0 * (1 - 2 * 1.5e-5) ** 2) < 0.05
    assert np.allclose(e[0], e[0][::-1, ::-1])
