"""Oracle-driven closed loop on the seeded SCAO scenarios (test helper).

The oracle closes the loop: frame k is generated from the residual slopes
turbulence_k - D c_{k-1}, then the oracle computes s_k, a_k, c_k.  The raw
frames are recorded so the HIP path can replay exactly the same pixels.
"""
from __future__ import annotations

import numpy as np

import oracle


def oracle_closed_loop(sc, n_frames: int, k0: int = 0):
    cfg = sc.cfg
    fo = oracle.FrameOracle(sc.mask, cfg.n_pix, sc.dark, sc.flat, cfg.threshold, sc.control_matrix,
                            cfg.gain, cfg.leak)
    h = cfg.frame_side
    frames = np.empty((n_frames, h, h), dtype=np.uint16)
    rec = {"counts": [], "slopes": [], "recon": [], "cmd": []}
    c = np.zeros(sc.n_act)
    for i in range(n_frames):
        k = k0 + i
        frames[i] = sc.frame(k, sc.residual_slopes(k, c if i > 0 else None))
        out = fo(frames[i], c)
        c = out["cmd"]
        for key in rec:
            rec[key].append(out[key])
    return frames, {key: np.stack(v) for key, v in rec.items()}


def oracle_closed_loop_multi(sc, n_frames: int, R=None, k0: int = 0):
    """Closed loop of a multi-sensor scenario; frame sets [n_frames, elements] and the oracle's record."""
    cfg = sc.cfg
    R = sc.control_matrix if R is None else R
    sets, rec = [], {"counts": [], "slopes": [], "recon": [], "cmd": []}
    c = np.zeros(sc.n_act)
    for i in range(n_frames):
        k = k0 + i
        frames = sc.frames(k, sc.residual_slopes(k, c if i > 0 else None))
        out = oracle.rtc_frame_multi(frames, sc.sensors, sc.darks, sc.flats, sc.thresholds, R, c, cfg.gain,
                                     cfg.leak)
        c = out["cmd"]
        sets.append(np.concatenate([f.ravel() for f in frames]))
        for key in rec:
            rec[key].append(out[key])
    return np.stack(sets), {key: np.stack(v) for key, v in rec.items()}
