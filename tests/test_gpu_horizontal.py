"""Persistent frames in the horizontal split (RTC_FRAMES_HORIZONTAL): every
workgroup multiplies its own subapertures' slopes into its own matrix columns,
kept on chip, and the partial actuator vectors are added by their owners.

Parity against the FP64 oracle (the float32 gates of the other modes; reduced
formats against the oracle run with the dequantised matrix), including one
launch of 1000 oracle-driven ELT closed-loop frames checked frame by frame."""
import numpy as np
import pytest

from _closedloop import oracle_closed_loop
from _gpu_helpers import _ctx_for, _dev, _gpu_batch, check_parity, dequantised_ref
from aosim import ELT, TINY, Scenario, geometry

torch = pytest.importorskip("torch")
from paper_1805_07254_amd import rtc  # noqa: E402

pytestmark = pytest.mark.gpu
H = rtc.RTC_FRAMES_HORIZONTAL


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rtc.load_library()


@pytest.fixture(scope="module")
def tiny_loop():
    sc = Scenario(TINY)
    return (sc,) + oracle_closed_loop(sc, 300)


@pytest.fixture(scope="module")
def elt_long():
    sc = Scenario(ELT)
    print("generating 1000 oracle-driven ELT closed-loop frames", flush=True)
    return (sc,) + oracle_closed_loop(sc, 1000)


def _ref_for(ref, sc, fmt):
    if fmt == "f32":
        return ref
    return dequantised_ref(ref, sc.control_matrix, fmt, sc.cfg.gain, sc.cfg.leak)[0]


@pytest.mark.parametrize("fmt", ["f32", "f16", "bf16", "fp8e4m3"])
def test_horizontal_tiny_closed_loop_matches_oracle(tiny_loop, fmt):
    sc, frames, ref = tiny_loop
    with _ctx_for(sc, cm_dtype=fmt) as ctx:
        rtc.rtc_set_frame_mode(ctx, H)
        assert rtc.rtc_get_frame_mode(ctx) == H
        gpu = _gpu_batch(ctx, frames, ts=True)
        rtc.rtc_sync_check(ctx)
        state = rtc.rtc_get_state(ctx)
    assert np.array_equal(state, gpu["cmd"][-1])
    ts = gpu["ts"]
    assert np.all(ts[:, 1] > ts[:, 0]) and np.all(ts[1:, 0] >= ts[:-1, 0])
    check_parity(gpu, _ref_for(ref, sc, fmt), sc.cfg.gain, sc.cfg.leak, what=f"tiny horizontal {fmt}")


def test_horizontal_elt_1000_frames_in_one_launch_match_oracle_every_frame(elt_long):
    # the timed configuration: ELT FP32, one persistent horizontal launch
    sc, frames, ref = elt_long
    with _ctx_for(sc) as ctx:
        rtc.rtc_set_frame_mode(ctx, H)
        gpu = _gpu_batch(ctx, frames, ts=True)
        rtc.rtc_sync_check(ctx)
    assert np.array_equal(gpu["counts"].astype(np.int64), ref["counts"])
    check_parity(gpu, ref, sc.cfg.gain, sc.cfg.leak, what="ELT horizontal, 1000 frames")


def test_persistent_row_split_elt_1000_frames_match_oracle_every_frame(elt_long):
    sc, frames, ref = elt_long
    with _ctx_for(sc) as ctx:
        rtc.rtc_set_frame_mode(ctx, rtc.RTC_FRAMES_PERSISTENT)
        gpu = _gpu_batch(ctx, frames)
        rtc.rtc_sync_check(ctx)
    check_parity(gpu, ref, sc.cfg.gain, sc.cfg.leak, what="ELT persistent row split, 1000 frames")


@pytest.mark.parametrize("fmt", ["f16", "bf16", "fp8e4m3"])
def test_horizontal_elt_reduced_formats_match_dequantised_oracle(elt_long, fmt):
    sc, frames, ref = elt_long
    n = 6
    with _ctx_for(sc, cm_dtype=fmt) as ctx:
        rtc.rtc_set_frame_mode(ctx, H)
        gpu = _gpu_batch(ctx, frames[:n])
        rtc.rtc_sync_check(ctx)
    sub = {k: v[:n] for k, v in ref.items()}
    check_parity(gpu, _ref_for(sub, sc, fmt), sc.cfg.gain, sc.cfg.leak, what=f"ELT horizontal {fmt}")


def test_horizontal_is_deterministic_and_batches_compose(tiny_loop):
    sc, frames, ref = tiny_loop
    with _ctx_for(sc) as ctx:
        rtc.rtc_set_frame_mode(ctx, H)
        whole = _gpu_batch(ctx, frames[:40])
        rtc.rtc_reset(ctx)
        again = _gpu_batch(ctx, frames[:40])
        rtc.rtc_reset(ctx)
        a = _gpu_batch(ctx, frames[:17])
        b = _gpu_batch(ctx, frames[17:40])
        rtc.rtc_sync_check(ctx)
    for key in whole:
        assert np.array_equal(whole[key], again[key]), key
    assert np.array_equal(np.concatenate([a["cmd"], b["cmd"]]), whole["cmd"])


def test_horizontal_matrix_reload_rebuilds_the_layout(tiny_loop):
    sc, frames, ref = tiny_loop
    R2 = (sc.control_matrix * np.float32(0.5)).astype(np.float32)
    with _ctx_for(sc) as ctx:
        rtc.rtc_set_frame_mode(ctx, H)
        _gpu_batch(ctx, frames[:3])
        rtc.rtc_reset(ctx)
        rtc.rtc_load_cmat(ctx, R2)
        got = _gpu_batch(ctx, frames[:3])
        rtc.rtc_reset(ctx)
        rtc.rtc_set_frame_mode(ctx, rtc.RTC_FRAMES_PER_LAUNCH)
        per = _gpu_batch(ctx, frames[:3])
    a_ref = per["slopes"].astype(np.float64) @ R2.astype(np.float64).T
    assert np.abs(got["recon"] - a_ref).max() <= 1e-5 * np.abs(a_ref).max()
    assert np.abs(got["cmd"] - per["cmd"]).max() <= 1e-5 * np.abs(per["cmd"]).max()


def test_horizontal_expired_wait_is_reported(tiny_loop):
    sc, frames, ref = tiny_loop
    with _ctx_for(sc) as ctx:
        rtc.rtc_set_frame_mode(ctx, H, spin_limit=1)
        _gpu_batch(ctx, np.concatenate([frames] * 2))
        with pytest.raises(rtc.RtcError) as ei:
            rtc.rtc_sync_check(ctx)
        assert ei.value.status == rtc.RTC_E_DEVICE
        with pytest.raises(rtc.RtcError) as ei:
            _gpu_batch(ctx, frames[:2])
        assert ei.value.status == rtc.RTC_E_STATE
        rtc.rtc_reset(ctx)
        rtc.rtc_set_frame_mode(ctx, H)
        good = _gpu_batch(ctx, frames[:20])
        rtc.rtc_sync_check(ctx)
    check_parity(good, {k: v[:20] for k, v in ref.items()}, sc.cfg.gain, sc.cfg.leak, what="horizontal after abort")


def test_horizontal_stage_trace_is_ordered(tiny_loop):
    sc, frames, ref = tiny_loop
    F, G = 12, 256
    trace = torch.zeros(F * G * 8, dtype=torch.int64, device="cuda:0")
    with _ctx_for(sc) as ctx:
        rtc.rtc_set_frame_mode(ctx, H)
        rtc.rtc_set_trace(ctx, trace, F, G)
        _gpu_batch(ctx, frames[:F])
        rtc.rtc_sync_check(ctx)
    t = trace.cpu().numpy().reshape(F, G, 8)
    # start, slopes, partial vector published, stores complete, arrival, barrier passed, loaded, commands
    order = [0, 1, 4, 6, 7, 2, 3, 5]
    assert np.all(t > 0)
    for a, b in zip(order[:-1], order[1:]):
        assert np.all(t[:, :, b] >= t[:, :, a]), (a, b)


def test_horizontal_unsupported_shapes_are_refused():
    for n_pix in (3, 32):                           # odd tiles (no pixel pairs), tiles too wide
        mask = np.ones((4, 4), np.uint8)
        with rtc.rtc_init(mask, n_pix, 5) as ctx:
            with pytest.raises(rtc.RtcError) as ei:
                rtc.rtc_set_frame_mode(ctx, H)
            assert ei.value.status == rtc.RTC_E_UNSUPPORTED
            assert rtc.rtc_get_frame_mode(ctx) == rtc.RTC_FRAMES_PER_LAUNCH


def test_horizontal_small_odd_shapes_match_per_launch():
    # few subapertures (empty workgroups), rows per owner 0 or 1, a ragged tail
    rng = np.random.default_rng(21)
    for n_sub, n_pix, n_act in ((3, 4, 7), (9, 6, 300), (23, 8, 600)):
        mask = geometry.subaperture_mask(n_sub, 0.2)
        nv = int(mask.sum())
        Hh = n_sub * n_pix
        frames = (rng.poisson(6.0, size=(4, Hh, Hh)) + 98).astype(np.uint16)
        frames[:, ::3, ::2] += rng.integers(0, 200, size=frames[:, ::3, ::2].shape).astype(np.uint16)
        dark = (100 + rng.standard_normal((Hh, Hh))).astype(np.float32)
        flat = (1 + 0.02 * rng.standard_normal((Hh, Hh))).astype(np.float32)
        R = (rng.standard_normal((n_act, 2 * nv)) / np.sqrt(2 * nv)).astype(np.float32)
        out = {}
        for mode in (rtc.RTC_FRAMES_PER_LAUNCH, H):
            with rtc.rtc_init(mask, n_pix, n_act) as ctx:
                rtc.rtc_load_calib(ctx, dark, flat, 3.0)
                rtc.rtc_load_cmat(ctx, R)
                rtc.rtc_set_frame_mode(ctx, mode)
                out[mode] = _gpu_batch(ctx, frames)
                rtc.rtc_sync_check(ctx)
        a, b = out[rtc.RTC_FRAMES_PER_LAUNCH], out[H]
        assert np.array_equal(a["counts"], b["counts"]) and np.array_equal(a["slopes"], b["slopes"])
        for key in ("recon", "cmd"):
            assert np.abs(a[key] - b[key]).max() <= 1e-5 * np.abs(a[key]).max(), (n_sub, key)
