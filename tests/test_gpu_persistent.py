"""Persistent frame batches (one cooperative launch, one grid barrier per frame)."""
import numpy as np
import pytest

import oracle
from _closedloop import oracle_closed_loop
from _gpu_helpers import _ctx_for, _dev, _gpu_batch, check_parity
from aosim import ELT, TINY, Scenario, geometry

torch = pytest.importorskip("torch")
from paper_1805_07254_amd import rtc  # noqa: E402

pytestmark = pytest.mark.gpu


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
def elt_loop():
    sc = Scenario(ELT)
    return (sc,) + oracle_closed_loop(sc, 5)


def _both_modes(sc, frames, fmt):
    with _ctx_for(sc, cm_dtype=fmt) as ctx:
        per = _gpu_batch(ctx, frames, ts=True)
        rtc.rtc_reset(ctx)
        rtc.rtc_set_frame_mode(ctx, rtc.RTC_FRAMES_PERSISTENT)
        pers = _gpu_batch(ctx, frames, ts=True)
        rtc.rtc_sync_check(ctx)
        state = rtc.rtc_get_state(ctx)
    return per, pers, state


@pytest.mark.parametrize("fmt", ["f32", "f16", "bf16", "fp8e4m3"])
@pytest.mark.parametrize("which", ["tiny", "elt"])
def test_persistent_batch_is_bitwise_identical_to_per_launch(which, fmt, request):
    sc, frames, ref = request.getfixturevalue(f"{which}_loop")
    per, pers, state = _both_modes(sc, frames, fmt)
    for key in ("counts", "slopes", "recon", "cmd"):
        assert np.array_equal(per[key], pers[key]), f"{which} {fmt}: {key} differs"
    assert np.array_equal(state, pers["cmd"][-1])
    ts = pers["ts"]
    # frame f+1's calibration may start while other workgroups still finish frame f,
    # so only starts, ends and each frame's own span are ordered
    assert np.all(ts[:, 1] > ts[:, 0])
    assert np.all(ts[1:, 0] >= ts[:-1, 0]) and np.all(ts[1:, 1] >= ts[:-1, 1])
    if fmt == "f32":
        check_parity(pers, ref, sc.cfg.gain, sc.cfg.leak, what=f"{which} persistent")


def test_persistent_batch_continues_from_state_and_chunks_compose(tiny_loop):
    sc, frames, ref = tiny_loop
    with _ctx_for(sc) as ctx:
        rtc.rtc_set_frame_mode(ctx, rtc.RTC_FRAMES_PERSISTENT)
        whole = _gpu_batch(ctx, frames[:40])
        rtc.rtc_reset(ctx)
        a = _gpu_batch(ctx, frames[:17])
        b = _gpu_batch(ctx, frames[17:40])
        rtc.rtc_sync_check(ctx)
    assert np.array_equal(np.concatenate([a["cmd"], b["cmd"]]), whole["cmd"])


def test_expired_barrier_wait_is_reported_and_cleared(tiny_loop):
    # A spin limit of one poll makes the kernel's own bounded waits give up; the
    # batch winds down normally and the host is told.
    sc, frames, ref = tiny_loop
    with _ctx_for(sc) as ctx:
        rtc.rtc_set_frame_mode(ctx, rtc.RTC_FRAMES_PERSISTENT, spin_limit=1)
        _gpu_batch(ctx, np.concatenate([frames] * 2))
        with pytest.raises(rtc.RtcError) as ei:
            rtc.rtc_sync_check(ctx)
        assert ei.value.status == rtc.RTC_E_DEVICE and "bounded wait" in str(ei.value)
        rtc.rtc_sync_check(ctx)                     # cleared
        rtc.rtc_set_frame_mode(ctx, rtc.RTC_FRAMES_PERSISTENT)
        # the state is undefined after the failed batch: frames are refused until a reset
        with pytest.raises(rtc.RtcError) as ei:
            _gpu_batch(ctx, frames[:2])
        assert ei.value.status == rtc.RTC_E_STATE
        rtc.rtc_reset(ctx)
        good = _gpu_batch(ctx, frames[:20])
        rtc.rtc_sync_check(ctx)
    check_parity(good, {k: v[:20] for k, v in ref.items()}, sc.cfg.gain, sc.cfg.leak, what="after abort")


@pytest.mark.parametrize("fmt", ["f32", "bf16"])
def test_long_slope_vectors_run_in_panels_identically_in_both_modes(fmt):
    # 19,000+ slopes exceed 8 wavefronts' register slices: two slope panels
    rng = np.random.default_rng(8)
    mask = geometry.subaperture_mask(110, 0.0)
    nv = int(mask.sum())
    H = 110
    frames = rng.integers(95, 200, size=(3, H, H)).astype(np.uint16)
    dark = np.full((H, H), 100.0, np.float32)
    flat = np.ones((H, H), np.float32)
    R = (rng.standard_normal((300, 2 * nv)) / 100).astype(np.float32)
    out = []
    for mode in (rtc.RTC_FRAMES_PER_LAUNCH, rtc.RTC_FRAMES_PERSISTENT):
        with rtc.rtc_init(mask, 1, 300, cm_dtype=fmt) as ctx:
            rtc.rtc_load_calib(ctx, dark, flat, 3.0)
            rtc.rtc_load_cmat(ctx, R)
            rtc.rtc_set_frame_mode(ctx, mode)
            out.append(_gpu_batch(ctx, frames))
            rtc.rtc_sync_check(ctx)
    assert 2 * nv > 16384
    for key in out[0]:
        assert np.array_equal(out[0][key], out[1][key]), key
    # against the float64 product with the matrix as stored
    from oracle import quant
    Rq = R.astype(np.float64) if fmt == "f32" else quant.dequantize(*quant.encode(R, fmt), fmt)
    a_ref = out[0]["slopes"].astype(np.float64) @ Rq.T
    assert np.abs(out[0]["recon"] - a_ref).max() <= 1e-5 * np.abs(a_ref).max()


@pytest.mark.parametrize("blocks", [0, 64, 32])
def test_panel_calibration_blocks_in_lds_or_memory_match_per_launch(blocks):
    # slope panels with 10 x 10 pixel tiles: with the default grid a workgroup's
    # (dark, flat) blocks sit in LDS and its pixel loads of four passes are in
    # flight together; 64 workgroups keep the blocks in LDS without the tile
    # descriptor copy, 32 workgroups have more blocks than LDS holds and read
    # them from memory
    rng = np.random.default_rng(12)
    mask = geometry.subaperture_mask(110, 0.0)
    nv = int(mask.sum())
    n = 10
    H = 110 * n
    frames = rng.integers(95, 200, size=(3, H, H)).astype(np.uint16)
    dark = rng.uniform(95.0, 105.0, size=(H, H)).astype(np.float32)
    flat = rng.normal(1.0, 0.02, size=(H, H)).astype(np.float32)
    R = (rng.standard_normal((300, 2 * nv)) / 100).astype(np.float32)
    out = []
    for mode, tuning in ((rtc.RTC_FRAMES_PER_LAUNCH, None), (rtc.RTC_FRAMES_PERSISTENT, {"blocks": blocks})):
        with rtc.rtc_init(mask, n, 300, cm_dtype="bf16") as ctx:
            rtc.rtc_load_calib(ctx, dark, flat, 20.0)
            rtc.rtc_load_cmat(ctx, R)
            rtc.rtc_set_frame_mode(ctx, mode)
            out.append(_gpu_batch(ctx, frames, tuning=tuning))
            rtc.rtc_sync_check(ctx)
    assert 2 * nv > 16384
    for key in out[0]:
        assert np.array_equal(out[0][key], out[1][key]), key
    ref = oracle.rtc_frame(frames[0], mask, n, dark, flat, 20.0, np.zeros((300, 2 * nv)), np.zeros(300), 0.4)
    assert np.array_equal(out[0]["counts"][0].astype(np.int64), ref["counts"])
    assert np.abs(out[0]["slopes"][0] - ref["slopes"]).max() <= 1e-5 * max(np.abs(ref["slopes"]).max(), 0.1)


@pytest.mark.parametrize("n_pix,fmt,n_sub", [(7, "f32", 12), (20, "f32", 12), (20, "bf16", 12), (7, "bf16", 160)])
def test_odd_and_wide_tiles_match_the_per_launch_result_and_the_oracle(n_pix, fmt, n_sub):
    # odd tile sides (single-pixel loads), tiles wider than 16 pixels (32 lanes
    # per tile, run-time calibration choices) and, with 160 x 160 subapertures,
    # slope panels with 8-lane odd tiles
    rng = np.random.default_rng(40 + n_pix + n_sub)
    mask = geometry.subaperture_mask(n_sub, 0.2)
    nv = int(mask.sum())
    H = n_sub * n_pix
    frames = rng.integers(90, 400, size=(3, H, H)).astype(np.uint16)
    dark = rng.uniform(95.0, 105.0, size=(H, H)).astype(np.float32)
    flat = rng.normal(1.0, 0.02, size=(H, H)).astype(np.float32)
    n_act = 250
    R = (rng.standard_normal((n_act, 2 * nv)) / 100).astype(np.float32)
    out = []
    for mode in (rtc.RTC_FRAMES_PER_LAUNCH, rtc.RTC_FRAMES_PERSISTENT):
        with rtc.rtc_init(mask, n_pix, n_act, cm_dtype=fmt) as ctx:
            rtc.rtc_load_calib(ctx, dark, flat, 60.0)
            rtc.rtc_load_cmat(ctx, R)
            rtc.rtc_set_frame_mode(ctx, mode)
            out.append(_gpu_batch(ctx, frames))
            rtc.rtc_sync_check(ctx)
    if n_sub == 160:
        assert 2 * nv > 32768                       # beyond 8 wavefronts' BF16 slices: slope panels
    for key in out[0]:
        assert np.array_equal(out[0][key], out[1][key]), key
    ref = oracle.rtc_frame(frames[0], mask, n_pix, dark, flat, 60.0, np.zeros((1, 2 * nv)), np.zeros(1), 0.4)
    assert ref["counts"].min() < n_pix * n_pix and ref["counts"].max() > 0
    assert np.array_equal(out[0]["counts"][0].astype(np.int64), ref["counts"])
    assert np.abs(out[0]["slopes"][0] - ref["slopes"]).max() <= 1e-5 * max(np.abs(ref["slopes"]).max(), 0.1)


def test_unsupported_persistent_shape_runs_per_launch():
    # more than 512 actuator rows per compute unit: one launch pair per frame
    rng = np.random.default_rng(9)
    mask = np.ones((2, 2), np.uint8)
    n_act = 131_073 * 2
    frames = rng.integers(95, 200, size=(2, 8, 8)).astype(np.uint16)
    R = (rng.standard_normal((n_act, 8)) / 10).astype(np.float32)
    out = []
    for mode in (rtc.RTC_FRAMES_PER_LAUNCH, rtc.RTC_FRAMES_PERSISTENT):
        with rtc.rtc_init(mask, 4, n_act) as ctx:
            rtc.rtc_load_calib(ctx, np.full((8, 8), 100.0, np.float32), np.ones((8, 8), np.float32), 3.0)
            rtc.rtc_load_cmat(ctx, R)
            rtc.rtc_set_frame_mode(ctx, mode)
            out.append(_gpu_batch(ctx, frames))
            rtc.rtc_sync_check(ctx)
    for key in out[0]:
        assert np.array_equal(out[0][key], out[1][key])


def test_frame_mode_validation():
    with rtc.rtc_init(np.ones((2, 2), np.uint8), 2, 3) as ctx:
        for bad in [(3, 0), (-1, 0), (1, -5)]:
            with pytest.raises(rtc.RtcError) as ei:
                rtc.rtc_set_frame_mode(ctx, *bad)
            assert ei.value.status == rtc.RTC_E_ARG


@pytest.mark.parametrize("fmt", ["f32", "bf16", "fp8e4m3"])
@pytest.mark.parametrize("which", ["tiny", "elt"])
def test_row_grouping_leaves_every_row_sum_bitwise_unchanged(which, fmt, request):
    # rows_per_wave 1 reduces each row on its own; 2 and 4 reduce rows transposed
    # across lanes.  Every row must see the same addition tree either way.
    sc, frames, _ = request.getfixturevalue(f"{which}_loop")
    frames = frames[:3]
    outs = []
    with _ctx_for(sc, cm_dtype=fmt) as ctx:
        for rpw in (1, 2, 4):
            rtc.rtc_reset(ctx)
            outs.append(_gpu_batch(ctx, frames, tuning=dict(rows_per_wave=rpw)))
    for o in outs[1:]:
        assert np.array_equal(o["recon"], outs[0]["recon"]), f"{which} {fmt}: row sums depend on grouping"
        assert np.array_equal(o["cmd"], outs[0]["cmd"])


def test_stage_trace_of_every_traced_workgroup_is_ordered(tiny_loop):
    sc, frames, _ = tiny_loop
    F, NG = 6, 3
    with _ctx_for(sc) as ctx:
        rtc.rtc_set_frame_mode(ctx, rtc.RTC_FRAMES_PERSISTENT)
        tr = torch.zeros(F * NG * 8, dtype=torch.int64, device="cuda:0")
        rtc.rtc_set_trace(ctx, tr, F, NG)
        _gpu_batch(ctx, frames[:F + 2], ts=True)
        rtc.rtc_sync_check(ctx)
        t = tr.cpu().numpy().reshape(F, NG, 8)
        rtc.rtc_set_trace(ctx, None, 0)
        with pytest.raises(rtc.RtcError):
            rtc.rtc_set_trace(ctx, tr, F, 0)
    stages = t[:, :, :6]
    assert np.all(stages > 0), "a traced workgroup left a stage unstamped"
    assert np.all(np.diff(stages, axis=2) >= 0), "stages out of order"
    assert np.all(np.diff(stages[:, :, 0], axis=0) > 0), "frame starts out of order"
    # no workgroup passes frame f's barrier before every traced one has published
    assert np.all(stages[:, :, 2].min(axis=1) >= stages[:, :, 1].max(axis=1))
    assert np.all(t[:, :, 6] >= t[:, :, 1]) and np.all(t[:, :, 7] >= t[:, :, 6])
    assert np.all(t[:, :, 2] >= t[:, :, 7])


@pytest.mark.parametrize("n_frames", [1, 2, 3, 4, 7])
def test_end_stamps_of_short_batches(tiny_loop, n_frames):
    """Every frame's end stamp is reduced: during a later frame's barrier for
    all but the last two frames, by the last workgroup to finish for those."""
    sc, frames, _ = tiny_loop
    with _ctx_for(sc, cm_dtype="f32") as ctx:
        rtc.rtc_set_frame_mode(ctx, rtc.RTC_FRAMES_PERSISTENT)
        for _ in range(2):                          # a second batch reuses the stamp rows
            out = _gpu_batch(ctx, frames[:n_frames], ts=True)
            rtc.rtc_sync_check(ctx)
            ts = out["ts"]
            assert np.all(ts[:, 0] > 0) and np.all(ts[:, 1] > ts[:, 0])
            assert np.all(ts[1:, 0] >= ts[:-1, 0]) and np.all(ts[1:, 1] >= ts[:-1, 1])
