"""Learned predictive control around the real-time controller.

The integrator of Section 2.1 (Figure 3 (d)) acts one frame after it measures,
so under frozen flow it always corrects the turbulence of the previous frame
(servo lag).  A small network forecasts how the next frame's pseudo-open-loop
(POL) modal coefficients will change and the forecast change is fed forward
into the integrator, so the leading modes are corrected in the frame they
change.  The plain integrator is the fallback and the reference its residual
is judged against.

Everything the controller computes runs in the library's kernels (C ABI):
reconstruction and integrator (rtc_reconstruct_integrate), the network's
forward and backward passes and Adam (rtc_mlp_*), and the predictor step
(rtc_pred_step).  torch only holds device memory, and the plant simulation
(turbulence slopes minus the mirror's slopes D c, plus noise) stands in for
the telescope.  The training set (modal coefficients of the telemetry, their
change statistics and windows) is prepared offline on the host in NumPy.

Data flow of one frame k (slopes r_k measured with commands c_{k-1} applied):
    integrator:  c_k = c_{k-1} + g R r_k
    predictive:  m_k = P r_k + (P D) c_{k-1}                      (POL modes)
                 d_k = network(last normalised changes of m)      (forecast m_{k+1} - m_k)
                 c_k = c_{k-1} + g R (r_k + P^T d_k / g)          (the same integrator)
A zero forecast leaves the plain integrator, which is therefore the fallback.
"""
from __future__ import annotations

import numpy as np
import torch

from . import rtc


def make_context(sc, R: np.ndarray, gain: float, leak: float = 1.0) -> rtc.RtcContext:
    cfg = sc.cfg
    ctx = rtc.rtc_init(sc.mask, cfg.n_pix, R.shape[0], gain=gain, leak=leak)
    rtc.rtc_load_calib(ctx, sc.dark, sc.flat, cfg.threshold)
    rtc.rtc_load_cmat(ctx, np.ascontiguousarray(R, dtype=np.float32))
    return ctx


def run_loop(D: torch.Tensor, s_tur: torch.Tensor, noise: torch.Tensor, ctx: rtc.RtcContext,
             pred: "rtc.Predictor | None" = None) -> dict:
    """Closed loop over the frames of s_tur [F, n_slopes] (device float32).

    Plant: r_k = s_tur_k - D c_{k-1} + n_k.  Controller: the integrator of ctx,
    fed the predictor's slopes r' when ``pred`` is given.  Returns residuals r
    [F, n_slopes] and the commands c_{k-1} [F, n_act] the plant saw.
    """
    F, ns = s_tur.shape
    n_act = D.shape[1]
    rtc.rtc_reset(ctx)
    if pred is not None:
        pred.reset()
    dev = s_tur.device
    c_prev = torch.zeros(n_act, dtype=torch.float32, device=dev)
    c_new = torch.empty(n_act, dtype=torch.float32, device=dev)
    res = torch.empty((F, ns), dtype=torch.float32, device=dev)
    cmds = torch.empty((F, n_act), dtype=torch.float32, device=dev)
    pad = (ns + 15) // 16 * 16
    r = torch.zeros(pad, dtype=torch.float32, device=dev)
    r2 = torch.zeros(pad, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev) if dev.type == "cuda" else None
    for k in range(F):
        cmds[k] = c_prev
        torch.sub(s_tur[k], D @ c_prev, out=r[:ns])
        r[:ns] += noise[k]
        res[k] = r[:ns]
        if pred is None:
            rtc.rtc_reconstruct_integrate(ctx, r, c_new, stream=stream)
        else:
            pred.step(r, c_prev, r2, stream=stream)
            rtc.rtc_reconstruct_integrate(ctx, r2, c_new, stream=stream)
        c_prev, c_new = c_new, c_prev
    torch.cuda.synchronize(dev) if dev.type == "cuda" else None
    return {"residual": res, "cmd_prev": cmds}


# Training-set preparation is offline work on the host (NumPy, float64): it
# runs once on recorded telemetry, not in the frame, and feeds the library's
# training kernels through device copies of its results.

def _host(a) -> np.ndarray:
    return a.detach().cpu().numpy() if isinstance(a, torch.Tensor) else np.asarray(a)


def pol_modes(residual, cmd_prev, P, PD) -> np.ndarray:
    """[F, n_modes] POL modal coefficients of closed-loop telemetry (the
    predictor step's m_k = P r_k + (P D) c_{k-1}), float64 on the host."""
    r = _host(residual).astype(np.float64)
    c = _host(cmd_prev).astype(np.float64)
    return r @ _host(P).astype(np.float64).T + c @ _host(PD).astype(np.float64).T


def change_stats(m) -> tuple[np.ndarray, np.ndarray]:
    """Mean and (sample) std of the per-frame changes of the modes [F, n_modes],
    float32 as the predictor takes them."""
    dm = np.diff(_host(m).astype(np.float64), axis=0)
    return dm.mean(axis=0).astype(np.float32), dm.std(axis=0, ddof=1).astype(np.float32)


def windows(m, history: int, mean, std) -> tuple[np.ndarray, np.ndarray]:
    """Training pairs from one segment of modes m [F, n_modes]: inputs [F - 1 - history,
    history n_modes] (the last ``history`` normalised changes, oldest first) and
    targets (the next normalised change), float32 on the host."""
    mu = _host(mean).astype(np.float64)
    sd = _host(std).astype(np.float64)
    z = (np.diff(_host(m).astype(np.float64), axis=0) - mu) / sd
    n = z.shape[0] - history
    x = np.lib.stride_tricks.sliding_window_view(z, history, axis=0)[:n]    # [n, n_modes, history]
    x = np.ascontiguousarray(x.transpose(0, 2, 1).reshape(n, history * z.shape[1]), dtype=np.float32)
    return x, np.ascontiguousarray(z[history:], dtype=np.float32)


def to_device(a: np.ndarray, device) -> torch.Tensor:
    """A host array as a device float32 tensor (a copy; the training kernels read it)."""
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)


def init_params(n_in: int, n_hidden: int, n_out: int, seed: int):
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal((n_hidden, n_in)) / np.sqrt(n_in)).astype(np.float32),
            np.zeros(n_hidden, np.float32),
            (rng.standard_normal((n_out, n_hidden)) * 0.1 / np.sqrt(n_hidden)).astype(np.float32),
            np.zeros(n_out, np.float32)]


def train(net: rtc.MlpNet, x: torch.Tensor, y: torch.Tensor, epochs: int, batch: int, lr: float, seed: int,
          x_val: torch.Tensor | None = None, y_val: torch.Tensor | None = None, log=None) -> list:
    """Adam on mean-square forecast error with the library's kernels; returns per-epoch losses."""
    n = x.shape[0]
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float32, device=x.device)
    hist, step = [], 0
    for ep in range(epochs):
        order = torch.randperm(n, generator=g).to(x.device)
        tot, nb = 0.0, 0
        lr_ep = lr * (0.3 ** ep if ep >= 2 else 1.0)
        for b0 in range(0, n - batch + 1, batch):
            idx = order[b0:b0 + batch]
            xb, yb = x[idx].contiguous(), y[idx].contiguous()
            net.loss_grad(batch, xb, yb, loss)
            step += 1
            net.adam(lr_ep, step)
            if nb % 50 == 0:
                tot += float(loss.item())
            nb += 1
        rec = {"epoch": ep, "train_loss": tot / max(1, (nb + 49) // 50)}
        if x_val is not None:
            rec["val_loss"] = evaluate(net, x_val, y_val, batch)
        hist.append(rec)
        if log:
            log(f"epoch {ep}: {rec}")
    return hist


def evaluate(net: rtc.MlpNet, x: torch.Tensor, y: torch.Tensor, batch: int) -> float:
    """Mean-square forecast error of the network on (x, y), forward passes only."""
    out = torch.empty((batch, y.shape[1]), dtype=torch.float32, device=x.device)
    se, cnt = 0.0, 0
    for b0 in range(0, x.shape[0] - batch + 1, batch):
        net.forward(batch, x[b0:b0 + batch].contiguous(), out)
        se += float(((out - y[b0:b0 + batch]) ** 2).sum().item())
        cnt += out.numel()
    return se / max(1, cnt)


def residual_rms(res: torch.Tensor, skip: int) -> float:
    r = res[skip:].to(torch.float64)
    return float(torch.sqrt(torch.mean(r * r)).item())
