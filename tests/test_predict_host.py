"""Offline training-set preparation of the predictor (host NumPy): windows,
change statistics, modal coefficients and the KL basis against their
definitions."""
import numpy as np

from aosim.telemetry import kl_basis
from paper_1805_07254_amd import predict


def test_windows_are_the_last_changes_oldest_first():
    rng = np.random.default_rng(0)
    m = rng.standard_normal((30, 5))
    mean, std = predict.change_stats(m)
    dm = np.diff(m, axis=0)
    assert np.allclose(mean, dm.mean(axis=0), rtol=1e-6)
    assert np.allclose(std, dm.std(axis=0, ddof=1), rtol=1e-6)
    x, y = predict.windows(m, 3, mean, std)
    z = (dm - mean.astype(np.float64)) / std.astype(np.float64)
    assert x.shape == (26, 15) and y.shape == (26, 5)
    for i in range(x.shape[0]):
        assert np.allclose(x[i], np.concatenate([z[i], z[i + 1], z[i + 2]]), rtol=1e-6, atol=1e-7)
        assert np.allclose(y[i], z[i + 3], rtol=1e-6, atol=1e-7)


def test_pol_modes_is_p_r_plus_pd_c():
    rng = np.random.default_rng(1)
    r, c = rng.standard_normal((7, 12)), rng.standard_normal((7, 4))
    P, PD = rng.standard_normal((3, 12)), rng.standard_normal((3, 4))
    m = predict.pol_modes(r.astype(np.float32), c.astype(np.float32), P.astype(np.float32), PD.astype(np.float32))
    want = np.array([[sum(P[j, i] * np.float32(r[k, i]) for i in range(12)) for j in range(3)] for k in range(7)])
    want += np.array([[sum(PD[j, i] * np.float32(c[k, i]) for i in range(4)) for j in range(3)] for k in range(7)])
    assert np.allclose(m, want, rtol=1e-6, atol=1e-6)


def test_kl_basis_spans_the_leading_covariance_eigenvectors():
    rng = np.random.default_rng(2)
    S = rng.standard_normal((400, 12)) @ np.diag(np.arange(12, 0, -1.0)) @ np.linalg.qr(rng.standard_normal((12, 12)))[0]
    P = kl_basis(S, 4)
    assert P.shape == (4, 12) and P.dtype == np.float32
    assert np.allclose(P @ P.T, np.eye(4), atol=1e-5)
    w, v = np.linalg.eigh(np.cov(S.T))
    lead = v[:, ::-1][:, :4]
    assert np.allclose(np.abs(P.astype(np.float64) @ lead), np.eye(4), atol=1e-4)
