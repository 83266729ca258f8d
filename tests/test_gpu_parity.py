"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Gates (float32 path against the float64 oracle on the same raw frames):
  * threshold counts and index maps: bit-exact;
  * slopes, per frame: max |ds| <= 1e-5 * max(max|s_ref|, 0.1 px);
  * reconstruction, per frame: max |da| <= 1e-5 * max|a_ref|;
  * integrator, per step: max |c_k - (leak c_{k-1} + gain a_k_ref)| <= 1e-5 * max|.|,
    with c_{k-1} the GPU's own previous command (replayed recurrences drift like
    sqrt(k) rounding steps, so the trajectory itself is reported, not gated).
Exact-arithmetic inputs (integers, dyadic calibration, gain 0.5) are bit-exact.
"""
import math
import time

import numpy as np
import pytest

import oracle
from _cases import near_tie_pixels, out_of_domain_tie_pixels
from _closedloop import oracle_closed_loop
from aosim import ELT, TINY, Scenario, geometry

torch = pytest.importorskip("torch")
from paper_1805_07254_amd import rtc  # noqa: E402
from _gpu_helpers import TOL, _ctx_for, _dev, _gpu_batch, check_parity  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rtc.load_library()


# ------------------------------------------------------------------ workloads
@pytest.fixture(scope="module")
def tiny_loop():
    sc = Scenario(TINY)
    frames, ref = oracle_closed_loop(sc, TINY.frames)
    return sc, frames, ref


@pytest.fixture(scope="module")
def elt_loop():
    sc = Scenario(ELT)
    t = time.time()
    frames, ref = oracle_closed_loop(sc, 6)
    print(f"ELT oracle loop built in {time.time() - t:.1f}s", flush=True)
    return sc, frames, ref


@pytest.mark.parametrize("k_split", [1, 3])
def test_tiny_scao_closed_loop_replay(tiny_loop, k_split):
    sc, frames, ref = tiny_loop
    with _ctx_for(sc) as ctx:
        assert ctx.n_valid == 80 and ctx.n_act == 97
        gpu = _gpu_batch(ctx, frames, k_split)
    check_parity(gpu, ref, TINY.gain, TINY.leak, what=f"tiny k_split={k_split}")


@pytest.mark.parametrize("k_split", [1, 4])
def test_elt_scao_replay_full_size(elt_loop, k_split):
    sc, frames, ref = elt_loop
    with _ctx_for(sc) as ctx:
        assert ctx.n_valid == 3972 and ctx.n_act == 4421
        gpu = _gpu_batch(ctx, frames, k_split, ts=True)
    check_parity(gpu, ref, ELT.gain, ELT.leak, what=f"elt k_split={k_split}")
    ts = gpu["ts"]
    assert np.all(ts[:, 1] > ts[:, 0]) and np.all(ts[1:, 0] >= ts[:-1, 1])


SHAPES = ([dict(kernel=0, waves=w, rows_per_wave=rb, blocks=b) for w in (8, 16) for rb in (1, 2, 4, 8)
           for b in (0, 100)] +
          [dict(kernel=1, rows_per_wave=r, unroll=u, k_split=k) for (r, u) in
           [(1, 2), (1, 4), (1, 8), (2, 2), (2, 4), (2, 8), (4, 2), (4, 4)] for k in (1, 3)])


@pytest.mark.parametrize("tuning", SHAPES, ids=[str(t) for t in SHAPES])
def test_elt_every_mvm_shape_matches_oracle(elt_loop, tuning):
    sc, frames, ref = elt_loop
    with _ctx_for(sc) as ctx:
        gpu = _gpu_batch(ctx, frames[:2], tuning=tuning)
    check_parity(gpu, {k: v[:2] for k, v in ref.items()}, ELT.gain, ELT.leak, what=f"elt {tuning}")


def test_elt_replay_is_bitwise_deterministic(elt_loop):
    sc, frames, _ = elt_loop
    with _ctx_for(sc) as ctx:
        a = _gpu_batch(ctx, frames)
        rtc.rtc_reset(ctx)
        b = _gpu_batch(ctx, frames)
    for key in a:
        assert np.array_equal(a[key], b[key]), key


def test_single_frame_and_stage_calls_match_batch(tiny_loop):
    sc, frames, ref = tiny_loop
    with _ctx_for(sc) as ctx:
        batch = _gpu_batch(ctx, frames[:5])
        rtc.rtc_reset(ctx)
        for k in range(5):
            pix = _dev(frames[k])
            cmd = torch.empty(ctx.n_act, dtype=torch.float32, device="cuda:0")
            sl = torch.empty(ctx.n_slopes, dtype=torch.float32, device="cuda:0")
            cnt = torch.empty(ctx.n_valid, dtype=torch.int32, device="cuda:0")
            rtc.rtc_frame(ctx, pix, cmd, slopes=sl, counts=cnt)
            torch.cuda.synchronize()
            assert np.array_equal(cmd.cpu().numpy(), batch["cmd"][k])
            assert np.array_equal(sl.cpu().numpy(), batch["slopes"][k])
            assert np.array_equal(cnt.cpu().numpy(), batch["counts"][k])
        # stage calls: calibrate+centroid, then reconstruct+integrate from those slopes
        rtc.rtc_reset(ctx)
        sl = torch.empty(ctx.n_slopes, dtype=torch.float32, device="cuda:0")
        cnt = torch.empty(ctx.n_valid, dtype=torch.int32, device="cuda:0")
        cmd = torch.empty(ctx.n_act, dtype=torch.float32, device="cuda:0")
        rec = torch.empty(ctx.n_act, dtype=torch.float32, device="cuda:0")
        rtc.rtc_calibrate_centroid(ctx, _dev(frames[0]), sl, cnt)
        rtc.rtc_reconstruct_integrate(ctx, sl, cmd, rec)
        torch.cuda.synchronize()
        assert np.array_equal(sl.cpu().numpy(), batch["slopes"][0])
        assert np.array_equal(cmd.cpu().numpy(), batch["cmd"][0])
        assert np.array_equal(rec.cpu().numpy(), batch["recon"][0])
        # unaligned caller slope vector goes through the library's staging copy
        big = torch.zeros(ctx.n_slopes + 1, dtype=torch.float32, device="cuda:0")
        big[1:] = sl
        rtc.rtc_reset(ctx)
        rtc.rtc_reconstruct_integrate(ctx, big[1:].data_ptr(), cmd, rec)
        torch.cuda.synchronize()
        assert np.array_equal(cmd.cpu().numpy(), batch["cmd"][0])


# ----------------------------------------------------------- exact arithmetic
def _exact_setup(rng, n_sub=6, n_pix=4, obs=0.3, n_act=11):
    mask = geometry.subaperture_mask(n_sub, obs)
    H = n_sub * n_pix
    frame = rng.integers(90, 400, size=(H, H)).astype(np.uint16)
    dark = np.full((H, H), 100.0, np.float32)
    flat = rng.choice(np.array([0.5, 1.0, 2.0], np.float32), size=(H, H))
    return mask, frame, dark, flat


def test_integer_inputs_give_bit_exact_slopes_and_counts():
    rng = np.random.default_rng(21)
    mask, frame, dark, flat = _exact_setup(rng)
    nv = int(mask.sum())
    R = rng.integers(-3, 4, size=(11, 2 * nv)).astype(np.float32)
    for mode, name in [(rtc.RTC_THR_SUBTRACT, "subtract"), (rtc.RTC_THR_ZERO, "zero")]:
        ref = oracle.rtc_frame(frame, mask, 4, dark, flat, 2.0, R, np.zeros(11), 0.5, mode=name)
        with rtc.rtc_init(mask, 4, 11, thr_mode=mode, gain=0.5) as ctx:
            rtc.rtc_load_calib(ctx, dark, flat, 2.0)
            rtc.rtc_load_cmat(ctx, R)
            gpu = _gpu_batch(ctx, frame[None])
        assert np.array_equal(gpu["counts"][0], ref["counts"])
        assert np.array_equal(gpu["slopes"][0], ref["slopes"].astype(np.float32)), name


TUNINGS = [dict(), dict(waves=8, rows_per_wave=1), dict(waves=16, rows_per_wave=2, blocks=7),
           dict(kernel=1, k_split=1, rows_per_wave=1, unroll=8), dict(kernel=1, k_split=2),
           dict(kernel=1, k_split=7, rows_per_wave=4, unroll=2), dict(kernel=1, k_split=64)]


@pytest.mark.parametrize("tuning", TUNINGS, ids=[str(t) for t in TUNINGS])
def test_integer_matrix_and_slopes_give_bit_exact_commands(tuning):
    rng = np.random.default_rng(5)
    mask = geometry.subaperture_mask(12, 0.2)
    nv = int(mask.sum())
    n_act = 203
    R = rng.integers(-8, 9, size=(n_act, 2 * nv)).astype(np.float32)
    with rtc.rtc_init(mask, 2, n_act, gain=0.5) as ctx:
        rtc.rtc_load_calib(ctx, np.zeros((24, 24), np.float32), np.ones((24, 24), np.float32), 0.0)
        rtc.rtc_load_cmat(ctx, R)
        rtc.rtc_set_mvm_tuning(ctx, **tuning)
        c = np.zeros(n_act)
        cmd = torch.empty(n_act, dtype=torch.float32, device="cuda:0")
        rec = torch.empty(n_act, dtype=torch.float32, device="cuda:0")
        for _ in range(3):
            s = rng.integers(-20, 21, size=2 * nv).astype(np.float32)
            rtc.rtc_reconstruct_integrate(ctx, _dev(s), cmd, rec)
            a = oracle.reconstruct(R, s)
            c = oracle.integrate(c, a, 0.5)
            torch.cuda.synchronize()
            assert np.array_equal(rec.cpu().numpy().astype(np.float64), a)
            assert np.array_equal(cmd.cpu().numpy().astype(np.float64), c)


def test_threshold_near_ties_counts_bit_exact():
    raw, dark, flat, T = near_tie_pixels(seed=7, n_candidates=2000000, T=40000.0, flat_range=(0.7, 1.3))
    n = len(raw)
    assert n > 100
    n_pix, n_sub = 4, int(math.ceil(math.sqrt(n / 16)))
    H = n_sub * n_pix
    fr = np.zeros(H * H, np.uint16)
    dk = np.zeros(H * H, np.float32)
    fl = np.ones(H * H, np.float32)
    fr[:n], dk[:n], fl[:n] = raw, dark, flat
    fr, dk, fl = fr.reshape(H, H), dk.reshape(H, H), fl.reshape(H, H)
    mask = np.ones((n_sub, n_sub), np.uint8)
    R = np.eye(3, 2 * n_sub * n_sub, dtype=np.float32)
    ref = oracle.rtc_frame(fr, mask, n_pix, dk, fl, float(T[0]), R, np.zeros(3), 0.4)
    assert ref["counts"].sum() > 0
    with rtc.rtc_init(mask, n_pix, 3) as ctx:
        rtc.rtc_load_calib(ctx, dk, fl, float(T[0]))
        rtc.rtc_load_cmat(ctx, R)
        gpu = _gpu_batch(ctx, fr[None])
    assert np.array_equal(gpu["counts"][0].astype(np.int64), ref["counts"])
    check_parity(gpu, {k: v[None] for k, v in ref.items()}, 0.4, 1.0, what="near ties")


@pytest.mark.parametrize("mode", [rtc.RTC_FRAMES_PER_LAUNCH, rtc.RTC_FRAMES_PERSISTENT])
def test_threshold_ties_with_darks_outside_the_fast_domain_counts_bit_exact(mode):
    # tiny, subnormal and 2^60 darks at exact and near ties of T = 3: raw - dark
    # is not exact in float64, so the device's exact expansion decides
    raw, dark, flat = out_of_domain_tie_pixels(3.0)
    n = len(raw)
    n_pix = 4
    n_sub = int(math.ceil(math.sqrt(n / 4)))       # 4 constructed pixels per tile, the rest below T
    H = n_sub * n_pix
    fr = np.full((H, H), 100, np.uint16)
    dk = np.full((H, H), 100.0, np.float32)
    fl = np.ones((H, H), np.float32)
    for i in range(n):
        t = i // 4
        sy, sx = divmod(t, n_sub)
        r, c = sy * n_pix + (i % 4), sx * n_pix + (i % 4)
        fr[r, c], dk[r, c], fl[r, c] = raw[i], dark[i], flat[i]
    mask = np.ones((n_sub, n_sub), np.uint8)
    R = np.eye(3, 2 * n_sub * n_sub, dtype=np.float32)
    ref = oracle.rtc_frame(fr, mask, n_pix, dk, fl, 3.0, R, np.zeros(3), 0.4)
    assert 0 < ref["counts"].sum() < n
    with rtc.rtc_init(mask, n_pix, 3) as ctx:
        rtc.rtc_load_calib(ctx, dk, fl, 3.0)
        rtc.rtc_load_cmat(ctx, R)
        rtc.rtc_set_frame_mode(ctx, mode)
        gpu = _gpu_batch(ctx, fr[None])
        rtc.rtc_sync_check(ctx)
    assert np.array_equal(gpu["counts"][0].astype(np.int64), ref["counts"])
    check_parity(gpu, {k: v[None] for k, v in ref.items()}, 0.4, 1.0, what="out-of-domain dark ties")


# -------------------------------------------------------------- edge cases
EDGE = [
    # n_sub, n_pix, obs, n_act, mode, k_split, ref, leak, clamp
    (5, 1, 0.0, 3, "subtract", 1, False, 1.0, None),
    (7, 3, 0.3, 13, "zero", 2, True, 0.99, None),
    (9, 32, 0.0, 37, "subtract", 1, False, 1.0, (-0.05, 0.05)),
    (13, 10, 0.28, 201, "subtract", 64, True, 1.0, None),
    (3, 6, 0.0, 1, "zero", 3, False, 0.5, None),
    (3, 5, 0.0, 9, "subtract", 1, False, 1.0, None),      # 9 subapertures: odd, padded slope vector
    (4, 8, 0.0, 70001, "subtract", 1, False, 1.0, None),  # many actuators, 32 slopes
    (6, 8, 0.0, 40, "none", 1, True, 1.0, None),           # no threshold applied
    (11, 4, 0.2, 57, "none", 4, False, 0.9, None),
]


@pytest.mark.parametrize("idx", range(len(EDGE)), ids=[f"edge{i}" for i in range(len(EDGE))])
def test_edge_configurations(idx):
    case = EDGE[idx]
    n_sub, n_pix, obs, n_act, mode, k_split, use_ref, leak, clamp = case
    rng = np.random.default_rng(1000 + idx)
    mask = geometry.subaperture_mask(n_sub, obs)
    nv = int(mask.sum())
    H = n_sub * n_pix
    F = 3
    frames = rng.poisson(8.0, size=(F, H, H)) + rng.integers(95, 106, size=(F, H, H))
    frames[:, ::2, ::3] += rng.integers(0, 300, size=frames[:, ::2, ::3].shape)
    frames = frames.astype(np.uint16)
    dark = (100 + rng.standard_normal((H, H))).astype(np.float32)
    flat = (1 + 0.02 * rng.standard_normal((H, H))).astype(np.float32)
    R = (rng.standard_normal((n_act, 2 * nv)) / np.sqrt(2 * nv)).astype(np.float32)
    ref_s = (0.1 * rng.standard_normal(2 * nv)).astype(np.float32) if use_ref else None
    c0 = (0.01 * rng.standard_normal(n_act)).astype(np.float32)
    lo, hi = clamp if clamp else (-math.inf, math.inf)
    mode_id = {"subtract": rtc.RTC_THR_SUBTRACT, "zero": rtc.RTC_THR_ZERO, "none": rtc.RTC_THR_NONE}[mode]
    with rtc.rtc_init(mask, n_pix, n_act, thr_mode=mode_id, gain=0.4, leak=leak, cmd_min=lo, cmd_max=hi) as ctx:
        rtc.rtc_load_calib(ctx, dark, flat, 3.0, ref_s)
        rtc.rtc_load_cmat(ctx, R)
        rtc.rtc_set_state(ctx, c0)
        gpu = _gpu_batch(ctx, frames, k_split)
        assert np.array_equal(rtc.rtc_get_state(ctx), gpu["cmd"][-1])
    c = c0.astype(np.float64)
    ref = {"counts": [], "slopes": [], "recon": [], "cmd": []}
    for k in range(F):
        out = oracle.rtc_frame(frames[k], mask, n_pix, dark, flat, 3.0, R, c, 0.4, leak, mode, ref_s, lo, hi)
        c = out["cmd"]
        for key in ref:
            ref[key].append(out[key])
    ref = {k: np.stack(v) for k, v in ref.items()}
    if clamp is None:
        check_parity(gpu, ref, 0.4, leak, c0=c0, what=str(case))
    else:
        assert np.array_equal(gpu["counts"].astype(np.int64), ref["counts"])
        assert np.all(gpu["cmd"] >= np.float32(lo)) and np.all(gpu["cmd"] <= np.float32(hi))
        pred = np.clip(leak * c0 + 0.4 * ref["recon"][0], lo, hi)
        assert np.abs(gpu["cmd"][0] - pred).max() <= TOL * np.abs(pred).max()


def test_empty_subapertures_and_zero_frames():
    mask = np.ones((3, 3), np.uint8)
    with rtc.rtc_init(mask, 4, 2) as ctx:
        dark = np.full((12, 12), 100.0, np.float32)
        rtc.rtc_load_calib(ctx, dark, np.ones((12, 12), np.float32), 5.0,
                           np.arange(18, dtype=np.float32) / 8)
        rtc.rtc_load_cmat(ctx, np.ones((2, 18), np.float32))
        frame = np.full((12, 12), 100, np.uint16)
        frame[5, 6] = 120                 # only subaperture 4 has a pixel above threshold
        gpu = _gpu_batch(ctx, frame[None])
        empty = torch.empty(0, dtype=torch.uint16, device="cuda:0")
        rtc.rtc_frame_batch(ctx, 0, empty, torch.empty(0, dtype=torch.float32, device="cuda:0"))
    counts = gpu["counts"][0]
    assert counts.tolist() == [0, 0, 0, 0, 1, 0, 0, 0, 0]
    s = gpu["slopes"][0]
    exp = -np.arange(18, dtype=np.float32) / 8
    exp[4] += 0.5          # column 2 of 4 -> +0.5 px
    exp[9 + 4] += -0.5     # row 1 of 4 -> -0.5 px
    assert np.array_equal(s, exp)


# -------------------------------------------------------------- API contract
def test_call_order_and_failed_loads_leave_state_intact():
    rng = np.random.default_rng(3)
    mask = geometry.subaperture_mask(6, 0.0)
    nv = int(mask.sum())
    H = 24
    frame = rng.integers(95, 300, size=(H, H)).astype(np.uint16)
    dark = (100 + rng.standard_normal((H, H))).astype(np.float32)
    flat = np.ones((H, H), np.float32)
    R = rng.standard_normal((5, 2 * nv)).astype(np.float32)
    with rtc.rtc_init(mask, 4, 5) as ctx:
        cmd = torch.empty(5, dtype=torch.float32, device="cuda:0")
        pix = _dev(frame)
        with pytest.raises(rtc.RtcError) as ei:
            rtc.rtc_frame(ctx, pix, cmd)
        assert ei.value.status == rtc.RTC_E_STATE
        rtc.rtc_load_calib(ctx, dark, flat, 3.0)
        rtc.rtc_load_cmat(ctx, R)
        rtc.rtc_frame(ctx, pix, cmd)
        first = cmd.cpu().numpy().copy()
        assert mask[3, 3] == 1          # pixel (12, 12) lies in an active subaperture
        bad = dark.copy()
        bad[12, 12] = np.nan
        with pytest.raises(rtc.RtcError) as ei:
            rtc.rtc_load_calib(ctx, bad, flat, 3.0)
        assert ei.value.status == rtc.RTC_E_NONFINITE
        # a dark outside the one-fma domain is accepted (decided exactly per launch)
        tiny = dark.copy()
        tiny[12, 12] = 1e-5
        rtc.rtc_load_calib(ctx, tiny, flat, 3.0)
        rtc.rtc_frame(ctx, pix, cmd)
        rtc.rtc_reset(ctx)
        rtc.rtc_load_calib(ctx, dark, flat, 3.0)
        # pixels outside the active subapertures are never read, so they are not checked
        corner = dark.copy()
        corner[0, 0] = np.nan
        assert mask[0, 0] == 0
        rtc.rtc_load_calib(ctx, corner, flat, 3.0)
        rtc.rtc_frame(ctx, pix, cmd)
        rtc.rtc_reset(ctx)
        with pytest.raises(rtc.RtcError) as ei:
            rtc.rtc_load_calib(ctx, dark, flat, -1.0)
        assert ei.value.status == rtc.RTC_E_ARG
        Rb = R.copy()
        Rb[2, 3] = np.inf
        with pytest.raises(rtc.RtcError) as ei:
            rtc.rtc_load_cmat(ctx, Rb)
        assert ei.value.status == rtc.RTC_E_NONFINITE
        with pytest.raises(rtc.RtcError) as ei:
            rtc.rtc_load_cmat(ctx, R[:, :-2])
        assert ei.value.status == rtc.RTC_E_ARG
        bad = [dict(kernel=1, k_split=65), dict(kernel=1, k_split=0), dict(kernel=1, rows_per_wave=3),
               dict(kernel=1, rows_per_wave=4, unroll=8), dict(kernel=1, unroll=16), dict(kernel=2),
               dict(waves=4), dict(rows_per_wave=9), dict(blocks=-1)]
        for bad_t in bad:
            with pytest.raises(rtc.RtcError) as ei:
                rtc.rtc_set_mvm_tuning(ctx, **bad_t)
            assert ei.value.status == rtc.RTC_E_ARG
        assert rtc.rtc_get_mvm_tuning(ctx) == rtc.TUNING_DEFAULT
        # the failed loads changed nothing: same frame from the same state gives the same command
        rtc.rtc_reset(ctx)
        assert np.all(rtc.rtc_get_state(ctx) == 0)
        rtc.rtc_frame(ctx, pix, cmd)
        assert np.array_equal(cmd.cpu().numpy(), first)
        # padded matrix rows (ld > n_slopes)
        Rp = np.zeros((5, 2 * nv + 3), np.float32)
        Rp[:, :2 * nv] = R
        Rp[:, 2 * nv:] = np.nan       # never read
        rtc.rtc_load_cmat(ctx, Rp, n_slopes=2 * nv)
        rtc.rtc_reset(ctx)
        rtc.rtc_frame(ctx, pix, cmd)
        assert np.array_equal(cmd.cpu().numpy(), first)
        assert rtc.rtc_wall_clock_khz(ctx) > 0


def test_probe_kernels_move_the_bytes():
    with rtc.rtc_init(np.ones((1, 1), np.uint8), 1, 1) as ctx:
        src = torch.arange(1 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.zeros_like(src)
        rtc.rtc_probe_copy(ctx, src, dst, src.numel() * 4)
        out = torch.zeros(1, dtype=torch.float32, device="cuda:0")
        rtc.rtc_probe_read(ctx, src, src.numel() * 4, out)
        torch.cuda.synchronize()
        assert torch.equal(src, dst) and out.item() == 0.0
