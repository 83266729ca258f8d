"""Pins of the predictor oracle against finite differences, closed forms and
library conversions (no GPU)."""
import math

import numpy as np
import pytest
import torch

from oracle import predictor as pr


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-20, 20, 20000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(pr.bf16(x), ref)


def test_gelu_closed_forms():
    assert pr.gelu(np.array([0.0]))[0] == 0.0
    x = np.linspace(-6, 6, 241)
    # GELU(x) - GELU(-x) = x (Phi(x) + Phi(-x) = 1)
    assert np.allclose(pr.gelu(x) - pr.gelu(-x), x, atol=1e-13)
    assert abs(pr.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15      # Phi(1)
    assert abs(pr.gelu(np.array([20.0]))[0] - 20.0) < 1e-12


def test_gelu_grad_is_the_derivative():
    z = np.linspace(-5, 5, 101)
    h = 1e-5
    fd = (pr.gelu(z + h) - pr.gelu(z - h)) / (2 * h)
    assert np.allclose(pr.gelu_grad(z), fd, atol=1e-9)


@pytest.mark.parametrize("seed", [0, 1])
def test_gradients_match_finite_differences(seed):
    rng = np.random.default_rng(seed)
    n_in, n_hid, n_out, B = 7, 5, 3, 4
    params = [rng.standard_normal((n_hid, n_in)), rng.standard_normal(n_hid) * 0.3,
              rng.standard_normal((n_out, n_hid)), rng.standard_normal(n_out) * 0.3]
    X = rng.standard_normal((B, n_in))
    T = rng.standard_normal((B, n_out))
    loss, grads, _ = pr.loss_grad(params, X, T, rounding=False)
    h = 1e-6
    for p, g in zip(params, grads):
        fd = np.zeros_like(p)
        for idx in np.ndindex(p.shape):
            old = p[idx]
            p[idx] = old + h
            lp, _, _ = pr.loss_grad(params, X, T, rounding=False)
            p[idx] = old - h
            lm, _, _ = pr.loss_grad(params, X, T, rounding=False)
            p[idx] = old
            fd[idx] = (lp - lm) / (2 * h)
        assert np.allclose(g, fd, rtol=1e-6, atol=1e-8)


def test_loss_is_the_mean_square():
    rng = np.random.default_rng(3)
    params = [rng.standard_normal((4, 6)), np.zeros(4), rng.standard_normal((2, 4)), np.zeros(2)]
    X = rng.standard_normal((5, 6))
    T = rng.standard_normal((5, 2))
    loss, _, f = pr.loss_grad(params, X, T, rounding=False)
    # brute force: every output by explicit sums
    Y = np.zeros((5, 2))
    for b in range(5):
        h = [pr.gelu(np.array([sum(params[0][j, i] * X[b, i] for i in range(6))]))[0] for j in range(4)]
        for o in range(2):
            Y[b, o] = sum(params[2][o, j] * h[j] for j in range(4))
    assert np.allclose(f["Y"], Y, atol=1e-12)
    assert abs(loss - np.mean((Y - T) ** 2)) < 1e-12


def test_adam_first_steps_closed_form():
    g = np.array([0.5, -2.0, 1e-3])
    theta0 = np.array([1.0, 1.0, 1.0])
    th, m, v = pr.adam(theta0, np.zeros(3), np.zeros(3), g, lr=0.1, b1=0.9, b2=0.999, eps=1e-8, t=1)
    # after one step m_hat = g, v_hat = g^2: theta moves by lr g / (|g| + eps)
    assert np.allclose(th, theta0 - 0.1 * g / (np.abs(g) + 1e-8), rtol=1e-14)
    # a constant gradient keeps m_hat = g and v_hat = g^2 at every step
    for t in range(2, 6):
        th, m, v = pr.adam(th, m, v, g, 0.1, 0.9, 0.999, 1e-8, t)
    assert np.allclose(th, theta0 - 5 * 0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_predictor_step_warm_up_and_forecast():
    rng = np.random.default_rng(4)
    nm, ns, na, hist, gain = 3, 8, 5, 2, 0.5
    P = np.linalg.qr(rng.standard_normal((ns, nm)))[0].T             # orthonormal rows
    PD = rng.standard_normal((nm, na))
    mean, std = rng.standard_normal(nm) * 0.1, 1.0 + rng.random(nm)
    params = [np.zeros((4, hist * nm)), np.zeros(4), np.zeros((nm, 4)), np.full(nm, 0.5)]
    st = {}
    ms = []
    for k in range(hist + 1):                      # history changes need history + 1 frames
        r, c0 = rng.standard_normal(ns), rng.standard_normal(na)
        r2, m, mhat, st = pr.predictor_step(params, st, r, c0, P, PD, mean, std, hist, gain, rounding=False)
        ms.append(m)
        assert np.allclose(m, P @ r + PD @ c0)
        if k < hist:                                # warm-up: no forecast, the plain integrator's slopes
            assert np.array_equal(mhat, m) and np.array_equal(r2, r)
    # zero weights: the network outputs b2 = 0.5, so the forecast change is 0.5 std + mean
    d = 0.5 * std + mean
    assert np.allclose(mhat, ms[-1] + d) and len(st["window"]) == hist
    assert np.allclose(st["window"][-1], (ms[-1] - ms[-2] - mean) / std)
    # the integrator's extra command for these slopes is g R P^T d / g = R P^T d
    assert np.allclose(P @ (r2 - r), d / gain)
