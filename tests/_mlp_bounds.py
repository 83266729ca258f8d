"""Element-wise error bounds of the device network against the float64 oracle (test helper).

The device accumulates products of bfloat16 operands in float32 (at most
1.5 K 2^-24 sum|a b| for K terms) and rounds some intermediates to bfloat16.
When the device's value of a quantity lies within e of the oracle's value x,
its bfloat16 rounding lies within dev(x, e) = max |bf16(x +- e) - bf16(x)| of
the oracle's (rounding is monotone), which covers roundings that land on the
other side of a midpoint.  The bounds below propagate these through the
forward and backward pass in the order the device computes them.
"""
import numpy as np

from oracle import predictor as pr

U = 2.0 ** -24


def dev(x, e):
    r = pr.bf16(x)
    return np.maximum(np.abs(pr.bf16(x - e) - r), np.abs(pr.bf16(x + e) - r))


def _acc(A, eA, B, eB, K):
    """Bound of |device A B - exact Ar Br| for rounded operands with errors eA, eB (A [m,k], B [k,n])."""
    Aa, Ba = np.abs(A) + eA, np.abs(B) + eB
    return 1.5 * K * U * (Aa @ Ba) + eA @ Ba + np.abs(A) @ eB


def forward_bounds(params, X, eX=0.0):
    W1, b1, W2, b2 = (np.asarray(p, np.float64) for p in params)
    f = pr.forward(params, X)
    Xr, W1r, W2r = f["Xr"], f["W1r"], f["W2r"]
    eXr = dev(np.asarray(X, np.float64), eX) if np.any(eX) else np.zeros_like(Xr)
    eZ1 = _acc(Xr, eXr, W1r.T, 0.0 * W1r.T, Xr.shape[1]) + U * (np.abs(b1) + np.abs(f["Z1"]))
    eH = 1.13 * eZ1 + 8 * U * (np.abs(f["H"]) + 1e-30)
    eHr = dev(f["H"], eH)
    eY = _acc(f["Hr"], eHr, W2r.T, 0.0 * W2r.T, f["Hr"].shape[1]) + U * (np.abs(b2) + np.abs(f["Y"]))
    return f, {"Z1": eZ1, "H": eH, "Hr": eHr, "Y": eY, "Xr": eXr}


def grad_bounds(params, X, T):
    f, e = forward_bounds(params, X)
    loss, grads, g = pr.loss_grad(params, X, T)
    B, n_out = g["Y"].shape
    edY = 2.0 * e["Y"] / (B * n_out) + 2 * U * np.abs(g["dY"])
    edYr = dev(g["dY"], edY)
    eW2 = _acc(g["dYr"].T, edYr.T, g["Hr"], e["Hr"], B)
    eb2 = edY.sum(axis=0) + 1.5 * B * U * np.abs(g["dY"]).sum(axis=0)
    edH = _acc(g["dYr"], edYr, g["W2r"], 0.0 * g["W2r"], n_out)
    gp = np.abs(pr.gelu_grad(g["Z1"]))
    edZ1 = edH * gp + np.abs(g["dH"]) * 0.8 * e["Z1"] + 4 * U * np.abs(g["dZ1"])
    edZ1r = dev(g["dZ1"], edZ1)
    eW1 = _acc(g["dZ1r"].T, edZ1r.T, g["Xr"], e["Xr"], B)
    eb1 = edZ1.sum(axis=0) + 1.5 * B * U * np.abs(g["dZ1"]).sum(axis=0)
    eloss = float(np.sum(2 * np.abs(g["Y"] - np.asarray(T, np.float64)) * e["Y"] + e["Y"] ** 2) / (B * n_out)) \
        + 4 * U * loss
    return loss, grads, (eW1, eb1, eW2, eb2), eloss, g
