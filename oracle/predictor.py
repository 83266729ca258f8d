"""FP64 oracle of the learned predictor (two-layer perceptron, Adam, modal step).

TEST INFRASTRUCTURE.  Only the test suite may import this module.  It shares no
code with the HIP kernels.

The paper has no learned component; this follows the design of the project's
predictor (a network forecasting the next frame's pseudo-open-loop modal
coefficients to cancel the integrator's servo lag):

    Z1 = X W1^T + b1,  H = GELU(Z1),  Y = H W2^T + b2,
    loss = mean over the batch and outputs of (Y - T)^2,
    GELU(z) = z Phi(z) (exact normal CDF), GELU'(z) = Phi(z) + z phi(z).

Precision reading (``rounding=True``, the device's choice): X, W1, W2, H and
the backward gradients dY and dZ1 are rounded to bfloat16 (nearest, ties to
even) where they enter a product; products and sums are float64 here.  With
``rounding=False`` everything is float64, which is what the finite-difference
pins check.

Gradients (chain rule):
    dY = 2 (Y - T) / (B n_out);  dW2 = dY^T H;  db2 = sum_b dY;
    dH = dY W2;  dZ1 = dH * GELU'(Z1);  dW1 = dZ1^T X;  db1 = sum_b dZ1.
Adam (Kingma & Ba): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
    theta -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

from .quant import round_to_format


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 value (ties to even), float64."""
    return round_to_format(np.asarray(x, dtype=np.float64), "bf16")


def gelu(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def _r(x, rounding):
    return bf16(x) if rounding else np.asarray(x, dtype=np.float64)


def forward(params, X, rounding: bool = True) -> dict:
    """Forward pass; params = (W1, b1, W2, b2) float32 masters."""
    W1, b1, W2, b2 = (np.asarray(p, dtype=np.float64) for p in params)
    Xr, W1r, W2r = _r(X, rounding), _r(W1, rounding), _r(W2, rounding)
    Z1 = Xr @ W1r.T + b1
    H = gelu(Z1)
    Hr = _r(H, rounding)
    Y = Hr @ W2r.T + b2
    return {"Xr": Xr, "W1r": W1r, "W2r": W2r, "Z1": Z1, "H": H, "Hr": Hr, "Y": Y}


def loss_grad(params, X, T, rounding: bool = True):
    """(loss, (dW1, db1, dW2, db2), forward intermediates)."""
    f = forward(params, X, rounding)
    T = np.asarray(T, dtype=np.float64)
    B, n_out = f["Y"].shape
    D = f["Y"] - T
    loss = float(np.sum(D * D) / (B * n_out))
    dY = 2.0 * D / (B * n_out)
    dYr = _r(dY, rounding)
    dW2 = dYr.T @ f["Hr"]
    db2 = dY.sum(axis=0)
    dH = dYr @ f["W2r"]
    dZ1 = dH * gelu_grad(f["Z1"])
    dZ1r = _r(dZ1, rounding)
    dW1 = dZ1r.T @ f["Xr"]
    db1 = dZ1.sum(axis=0)
    f.update({"dY": dY, "dYr": dYr, "dH": dH, "dZ1": dZ1, "dZ1r": dZ1r})
    return loss, (dW1, db1, dW2, db2), f


def adam(theta, m, v, g, lr, b1, b2, eps, t):
    """One Adam step; returns (theta, m, v) in float64."""
    theta, m, v, g = (np.asarray(a, dtype=np.float64) for a in (theta, m, v, g))
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    theta = theta - lr * (m / (1.0 - b1 ** t)) / (np.sqrt(v / (1.0 - b2 ** t)) + eps)
    return theta, m, v


def predictor_step(params, state, r, c_prev, P, PD, mean, std, history, gain, rounding=True):
    """One frame of the predictive feed-forward.

    m = P r + PD c_prev; from the second frame on the window (oldest first,
    ``history`` rows) gains the normalised change (m - m_prev - mean) / std;
    when it holds ``history`` changes the forecast change is
    d = network(window) * std + mean, otherwise d = 0; the slopes handed to
    the integrator are r' = r + P^T d / gain.  ``state`` is a dict with
    "window" (list) and "m_prev" (None at start).  Returns (r', m, m + d, state).
    """
    P, PD = np.asarray(P, dtype=np.float64), np.asarray(PD, dtype=np.float64)
    mean, std = np.asarray(mean, np.float64), np.asarray(std, np.float64)
    r = np.asarray(r, np.float64)
    m = P @ r + PD @ np.asarray(c_prev, np.float64)
    window = list(state.get("window", []))
    if state.get("m_prev") is not None:
        window = (window + [(m - state["m_prev"] - mean) / std])[-history:]
    if len(window) == history:
        d = forward(params, np.concatenate(window)[None, :], rounding)["Y"][0] * std + mean
    else:
        d = np.zeros_like(m)
    r_out = r + P.T @ d / float(np.float32(gain))
    return r_out, m, m + d, {"window": window, "m_prev": m}
