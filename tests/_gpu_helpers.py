"""Shared helpers of the GPU parity tests (device transfers, batch replay, gates)."""
import numpy as np
import torch

import oracle
from oracle import quant
from paper_1805_07254_amd import rtc

TOL = 1e-5


def _dev(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint16:          # move the bits as int16, then view as uint16
        return torch.from_numpy(a.view(np.int16)).to("cuda:0").view(torch.uint16)
    return torch.from_numpy(a).to("cuda:0")


def _gpu_batch(ctx, frames, k_split=1, ts=False, tuning=None):
    F = frames.shape[0]
    pix = _dev(frames.reshape(F, -1))
    cmd = torch.empty(F * ctx.n_act, dtype=torch.float32, device="cuda:0")
    slopes = torch.empty(F * ctx.n_slopes, dtype=torch.float32, device="cuda:0")
    recon = torch.empty(F * ctx.n_act, dtype=torch.float32, device="cuda:0")
    counts = torch.empty(F * ctx.n_valid, dtype=torch.int32, device="cuda:0")
    tst = torch.zeros(2 * F, dtype=torch.int64, device="cuda:0") if ts else None
    if tuning is not None:
        rtc.rtc_set_mvm_tuning(ctx, **tuning)
    elif k_split > 1:
        rtc.rtc_set_mvm_tuning(ctx, kernel=rtc.RTC_MVM_STREAMED, k_split=k_split, rows_per_wave=2)
    else:
        rtc.rtc_set_mvm_tuning(ctx)
    rtc.rtc_frame_batch(ctx, F, pix, cmd, slopes, recon, counts, tst)
    torch.cuda.synchronize()
    out = {"cmd": cmd.cpu().numpy().reshape(F, -1), "slopes": slopes.cpu().numpy().reshape(F, -1),
           "recon": recon.cpu().numpy().reshape(F, -1), "counts": counts.cpu().numpy().reshape(F, -1)}
    if ts:
        out["ts"] = tst.cpu().numpy().reshape(F, 2)
    return out


def check_parity(gpu, ref, gain, leak, c0=None, what=""):
    g, lam = float(np.float32(gain)), float(np.float32(leak))
    F = ref["cmd"].shape[0]
    assert np.array_equal(gpu["counts"].astype(np.int64), ref["counts"]), f"{what}: counts differ"
    worst = {"s": 0.0, "a": 0.0, "c": 0.0}
    for k in range(F):
        s_ref = ref["slopes"][k]
        ds = np.abs(gpu["slopes"][k].astype(np.float64) - s_ref).max()
        tol_s = TOL * max(np.abs(s_ref).max(), 0.1)
        assert ds <= tol_s, f"{what} frame {k}: slopes off by {ds} > {tol_s}"
        a_ref = ref["recon"][k]
        da = np.abs(gpu["recon"][k].astype(np.float64) - a_ref).max()
        tol_a = TOL * np.abs(a_ref).max()
        assert da <= tol_a, f"{what} frame {k}: recon off by {da} > {tol_a}"
        c_prev = (gpu["cmd"][k - 1].astype(np.float64) if k else
                  (np.zeros_like(a_ref) if c0 is None else np.asarray(c0, np.float64)))
        pred = lam * c_prev + g * a_ref
        dc = np.abs(gpu["cmd"][k].astype(np.float64) - pred).max()
        tol_c = TOL * np.abs(pred).max()
        assert dc <= tol_c, f"{what} frame {k}: integrator off by {dc} > {tol_c}"
        worst["s"] = max(worst["s"], ds / tol_s * TOL)
        worst["a"] = max(worst["a"], da / tol_a * TOL if tol_a else 0.0)
        worst["c"] = max(worst["c"], dc / tol_c * TOL if tol_c else 0.0)
    drift = np.abs(gpu["cmd"][-1] - ref["cmd"][-1]).max() / max(np.abs(ref["cmd"][-1]).max(), 1e-30)
    print(f"{what}: worst relative errors {worst}, final command drift {drift:.2e}", flush=True)
    return worst


def _ctx_for(sc, **kw):
    cfg = sc.cfg
    ctx = rtc.rtc_init(sc.mask, cfg.n_pix, sc.n_act, gain=cfg.gain, leak=cfg.leak, **kw)
    rtc.rtc_load_calib(ctx, sc.dark, sc.flat, cfg.threshold)
    rtc.rtc_load_cmat(ctx, sc.control_matrix)
    return ctx


def dequantised_ref(ref, R, fmt, gain, leak):
    """The oracle record with the reconstruction redone with the dequantised
    matrix of a reduced storage format (slopes and counts unchanged)."""
    codes, scales = quant.encode(R, fmt)
    Rq = quant.dequantize(codes, scales, fmt)
    a = ref["slopes"] @ Rq.T
    c = np.zeros(R.shape[0])
    cmds = []
    for k in range(len(a)):
        c = oracle.integrate(c, a[k], gain, leak)
        cmds.append(c)
    return {"counts": ref["counts"], "slopes": ref["slopes"], "recon": a, "cmd": np.stack(cmds)}, Rq
