"""Long persistent runs at full size against the FP64 oracle: the benchmark's
launch (10,000 ELT frames in one persistent launch) and a closed loop of
1,000 ELT frames.

In the benchmark's launch the pixel frames are open-loop (no command feeds
back into them) and cycle through a ring of distinct frames, so the oracle computes
calibration, centroids and the reconstruction (Figure 3 (a)-(c)) once per
distinct frame.  Counts are compared bit for bit and slopes and
reconstructions within the per-frame tolerance for all 10,000 frames; the
integrator (Figure 3 (d)) is checked one step at a time and, over its whole
recursion, against the oracle's own recursion within an error bound built
from oracle values only.
"""
import numpy as np
import pytest

import oracle
from _closedloop import oracle_closed_loop
from _gpu_helpers import TOL, _ctx_for, check_parity
from aosim import ELT, Scenario

torch = pytest.importorskip("torch")
from paper_1805_07254_amd import rtc  # noqa: E402

pytestmark = pytest.mark.gpu

RING, FRAMES = 128, 10000
U32 = 2.0 ** -24                      # float32 unit roundoff


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rtc.load_library()


@pytest.fixture(scope="module")
def elt_ring():
    sc = Scenario(ELT)
    cfg = sc.cfg
    ring = np.stack([sc.frame(i, sc.turbulence_slopes(i)) for i in range(RING)])
    fo = oracle.FrameOracle(sc.mask, cfg.n_pix, sc.dark, sc.flat, cfg.threshold, sc.control_matrix, cfg.gain,
                            cfg.leak)
    zero = np.zeros(sc.n_act)
    outs = [fo(ring[i], zero) for i in range(RING)]
    ref = {k: np.stack([o[k] for o in outs]) for k in ("counts", "slopes", "recon")}
    return sc, ring, ref


def test_ten_thousand_elt_frames_in_one_persistent_launch(elt_ring):
    sc, ring, ref = elt_ring
    cfg = sc.cfg
    r16 = torch.from_numpy(ring.reshape(RING, -1).view(np.int16)).to("cuda:0")
    frames = r16[torch.arange(FRAMES, device="cuda:0") % RING].contiguous().view(torch.uint16)
    z = lambda n, dt=torch.float32: torch.zeros(n, dtype=dt, device="cuda:0")  # noqa: E731
    with _ctx_for(sc) as a, _ctx_for(sc) as b:
        for ctx in (a, b):
            rtc.rtc_set_mvm_tuning(ctx)
            rtc.rtc_set_frame_mode(ctx, rtc.RTC_FRAMES_PERSISTENT)
        cmd, slopes, recon = z(FRAMES * a.n_act), z(FRAMES * a.n_slopes), z(FRAMES * a.n_act)
        counts = z(FRAMES * a.n_valid, torch.int32)
        print(f"ELT persistent launch of {FRAMES} frames with every output", flush=True)
        rtc.rtc_frame_batch(a, FRAMES, frames, cmd, slopes, recon, counts)
        cmd_b = z(FRAMES * b.n_act)
        print(f"ELT persistent launch of {FRAMES} frames, commands only", flush=True)
        rtc.rtc_frame_batch(b, FRAMES, frames, cmd_b)
        torch.cuda.synchronize()
        rtc.rtc_sync_check(a)
        rtc.rtc_sync_check(b)
        # the benchmark's launch (commands only, no stamps) computes the same commands
        assert torch.equal(cmd, cmd_b)
        state = rtc.rtc_get_state(a)
    del frames, r16, cmd_b
    g_cmd = cmd.cpu().numpy().reshape(FRAMES, -1)
    g_s = slopes.cpu().numpy().reshape(FRAMES, -1)
    g_a = recon.cpu().numpy().reshape(FRAMES, -1)
    g_n = counts.cpu().numpy().reshape(FRAMES, -1)
    del cmd, slopes, recon, counts
    torch.cuda.empty_cache()
    assert np.array_equal(state, g_cmd[-1])

    g, lam = float(np.float32(cfg.gain)), float(np.float32(cfg.leak))
    c_ref = np.zeros(sc.n_act)          # the oracle's recursion
    bound = 0.0                         # bound on max |c_gpu - c_ref| after each frame
    c_prev = np.zeros(sc.n_act)         # the device's previous command (one-step check)
    worst = {"s": 0.0, "a": 0.0, "step": 0.0, "recursion": 0.0}
    for k in range(FRAMES):
        j = k % RING
        assert np.array_equal(g_n[k].astype(np.int64), ref["counts"][j]), f"frame {k}: counts differ"
        s_ref, a_ref = ref["slopes"][j], ref["recon"][j]
        ds = np.abs(g_s[k].astype(np.float64) - s_ref).max()
        tol_s = TOL * max(np.abs(s_ref).max(), 0.1)
        assert ds <= tol_s, f"frame {k}: slopes off by {ds} > {tol_s}"
        A = np.abs(a_ref).max()
        da = np.abs(g_a[k].astype(np.float64) - a_ref).max()
        assert da <= TOL * A, f"frame {k}: recon off by {da} > {TOL * A}"
        c_k = g_cmd[k].astype(np.float64)
        pred = lam * c_prev + g * a_ref
        dc = np.abs(c_k - pred).max()
        tol_c = TOL * np.abs(pred).max()
        assert dc <= tol_c, f"frame {k}: integrator step off by {dc} > {tol_c}"
        # recursion: e_k = lam e_(k-1) + g (a_gpu - a_ref) + rounding of the float32 step,
        # |a_gpu - a_ref| <= TOL A, rounding <= 2u (|c_k| + g A) with |c_k| <= |c_ref| + bound
        c_ref = oracle.integrate(c_ref, a_ref, cfg.gain, cfg.leak)
        bound = lam * bound + g * TOL * A + 2 * U32 * (np.abs(c_ref).max() + bound + g * A)
        dr = np.abs(c_k - c_ref).max()
        assert dr <= bound, f"frame {k}: command off the oracle's recursion by {dr} > {bound}"
        c_prev = c_k
        worst["s"] = max(worst["s"], ds / tol_s)
        worst["a"] = max(worst["a"], da / (TOL * A))
        worst["step"] = max(worst["step"], dc / tol_c if tol_c else 0.0)
        worst["recursion"] = max(worst["recursion"], dr / bound)
    print(f"{FRAMES} ELT frames: worst error / tolerance {worst}; final command "
          f"{np.abs(c_ref).max():.4g} max, off the oracle by {np.abs(g_cmd[-1] - c_ref).max():.3g}", flush=True)


def test_thousand_closed_loop_elt_frames_in_one_persistent_launch():
    # The oracle closes the loop (each frame made from the turbulence minus the
    # previous command), the device replays the recorded pixels in one
    # persistent launch; every frame is checked with the per-step gates, and
    # the commands against the oracle's own recursion within the bound above.
    sc = Scenario(ELT)
    F = 1000
    frames, ref = oracle_closed_loop(sc, F)
    pix = torch.from_numpy(frames.reshape(F, -1).view(np.int16)).to("cuda:0").view(torch.uint16)
    z = lambda n, dt=torch.float32: torch.zeros(n, dtype=dt, device="cuda:0")  # noqa: E731
    with _ctx_for(sc) as ctx:
        rtc.rtc_set_frame_mode(ctx, rtc.RTC_FRAMES_PERSISTENT)
        out = dict(cmd=z(F * ctx.n_act), slopes=z(F * ctx.n_slopes), recon=z(F * ctx.n_act),
                   counts=z(F * ctx.n_valid, torch.int32))
        print(f"ELT closed loop: persistent launch of {F} frames", flush=True)
        rtc.rtc_frame_batch(ctx, F, pix, out["cmd"], out["slopes"], out["recon"], out["counts"])
        torch.cuda.synchronize()
        rtc.rtc_sync_check(ctx)
    gpu = {k: v.cpu().numpy().reshape(F, -1) for k, v in out.items()}
    check_parity(gpu, ref, sc.cfg.gain, sc.cfg.leak, what=f"ELT closed loop, {F} persistent frames")
    g = float(np.float32(sc.cfg.gain))
    lam = float(np.float32(sc.cfg.leak))
    bound, worst = 0.0, 0.0
    for k in range(F):
        A = np.abs(ref["recon"][k]).max()
        c_ref = ref["cmd"][k]
        bound = lam * bound + g * TOL * A + 2 * U32 * (np.abs(c_ref).max() + bound + g * A)
        dr = np.abs(gpu["cmd"][k].astype(np.float64) - c_ref).max()
        assert dr <= bound, f"frame {k}: command off the oracle's recursion by {dr} > {bound}"
        worst = max(worst, dr / bound)
    print(f"closed loop: commands within {worst:.3f} of the recursion bound", flush=True)
