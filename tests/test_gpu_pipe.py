"""Pixel-stream processing on the GPU (Section 2.3.6, Figure 6; Section 3.2).

A camera workgroup lands the rows of each frame on a schedule; workers
calibrate, centroid and reconstruct their subapertures as their rows land,
and the partial actuator vectors are summed per actuator.  The results must
match the oracle like every other frame path, for any allocation, and the
time stamps must show the arrival constraints: no worker finishes before the
rows it needs have landed, no command is written before the last pixel, and
with pixel-stream processing the early workers finish before the last pixel.
"""
import numpy as np
import pytest

from _closedloop import oracle_closed_loop
from _gpu_helpers import _ctx_for, _dev, _gpu_batch, check_parity
from aosim import ELT, TINY, Scenario, geometry
import oracle

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
    return (sc,) + oracle_closed_loop(sc, 120)


@pytest.fixture(scope="module")
def elt_loop():
    sc = Scenario(ELT)
    return (sc,) + oracle_closed_loop(sc, 5)


def _pipe_run(ctx, frames, **cfg):
    rtc.rtc_pipe_setup(ctx, **cfg)
    info = rtc.rtc_pipe_info(ctx)
    F, P = frames.shape[0], info["n_workers"]
    pix = _dev(frames.reshape(F, -1))
    dev = dict(dtype=torch.float32, device="cuda:0")
    cmd, recon = torch.empty(F * ctx.n_act, **dev), torch.empty(F * ctx.n_act, **dev)
    slopes = torch.empty(F * ctx.n_slopes, **dev)
    counts = torch.empty(F * ctx.n_valid, dtype=torch.int32, device="cuda:0")
    cam = torch.zeros(4 * F, dtype=torch.int64, device="cuda:0")
    wk = torch.zeros(2 * F * P, dtype=torch.int64, device="cuda:0")
    print(f"pipe run: {F} frames, {P} workers, {cfg}", flush=True)
    rtc.rtc_pipe_run(ctx, F, pix, cmd, slopes, recon, counts, cam, wk)
    torch.cuda.synchronize()
    rtc.rtc_sync_check(ctx)
    return {"cmd": cmd.cpu().numpy().reshape(F, -1), "slopes": slopes.cpu().numpy().reshape(F, -1),
            "recon": recon.cpu().numpy().reshape(F, -1), "counts": counts.cpu().numpy().reshape(F, -1),
            "cam": cam.cpu().numpy().reshape(F, 4), "wk": wk.cpu().numpy().reshape(F, P, 2), "info": info}


def _check_arrival_order(sc, out, ratio, full, period_us, readout_us, khz, tail_rows=0):
    """Time stamps against the arrival schedule (device wall-clock ticks)."""
    cfg = sc.cfg
    cam, wk, P = out["cam"], out["wk"], out["info"]["n_workers"]
    H = out["info"]["image_rows"]
    tpu = khz / 1000.0
    t_row = readout_us * tpu / H
    assert np.all(cam[:, 1] >= cam[:, 0]) and np.all(cam[:, 2] >= cam[:, 1])
    assert np.all(cam[:, 2] - cam[:, 0] >= np.floor(readout_us * tpu) - 2), "last rows landed before schedule"
    assert np.all(np.diff(cam[:, 0]) >= np.floor(period_us * tpu) - 1)
    # rows each worker's subapertures need
    iy, _ = np.nonzero(sc.mask)
    need = (iy + 1) * cfg.n_pix
    n_tail = out["info"]["n_tail"]
    assert n_tail == np.count_nonzero(iy >= sc.mask.shape[0] - tail_rows)
    counts = rtc.rtc_pipe_allocation(len(need) - n_tail, P, ratio)
    last = np.cumsum(counts) - 1
    for b in np.nonzero(counts)[0]:
        nd = H if full else need[last[b]]
        earliest = cam[:, 0] + np.floor(nd * t_row) - 1
        assert np.all(wk[:, b, 0] >= earliest), f"worker {b} published before its rows landed"
    if full:
        assert np.all(wk[:, counts > 0, 0] >= cam[:, 2:3]), "a worker started before the whole frame landed"
    # every command needs every partial vector (and the tail), the last of which needs the last rows
    n_own = out["info"]["n_owners"]
    assert 1 <= n_own <= P and (sc.n_act + n_own - 1) // n_own <= 64
    assert np.all(wk[:, :n_own, 1] >= cam[:, 2:3])
    assert np.all(wk[:, :, 1] >= wk[:, :, 0])
    lat_us = (wk[:, :, 1].max(axis=1) - cam[:, 2]) / tpu
    early = (wk[1:, 0, 0] - cam[1:, 2]) / tpu
    print(f"ratio {ratio} full {full} tail {tail_rows}: latency last pixel -> last command {np.round(lat_us, 1)} us; "
          f"worker 0 partial vs last pixel {np.round(early, 1)} us; camera slip "
          f"{np.round(cam[:, 3] / tpu, 1)} us", flush=True)
    if not full:
        assert np.all(early < 0), "the first worker did not finish before the last pixel"
    return lat_us


@pytest.mark.parametrize("workers,ratio,full,tail", [(0, 1.0, False, 0), (0, 6.0, False, 0), (0, 1.0, True, 0),
                                                     (7, 3.0, False, 0), (2, 1.0, False, 0), (2, 1.0, True, 0),
                                                     (0, 4.0, False, 1), (7, 1.0, False, 2), (3, 2.0, True, 1),
                                                     (0, 1.0, False, 5)])
def test_pipe_matches_oracle_tiny(tiny_loop, workers, ratio, full, tail):
    sc, frames, ref = tiny_loop
    with _ctx_for(sc) as ctx:
        khz = rtc.rtc_wall_clock_khz(ctx)
        out = _pipe_run(ctx, frames, n_workers=workers, alloc_ratio=ratio, full_frame=full,
                        frame_period_us=200.0, readout_us=150.0, rows_per_packet=2, tail_rows=tail)
        state = rtc.rtc_get_state(ctx)
    check_parity(out, ref, sc.cfg.gain, sc.cfg.leak,
                 what=f"tiny pipe P={workers} ratio={ratio} full={full} tail={tail}")
    assert np.array_equal(state, out["cmd"][-1])
    _check_arrival_order(sc, out, ratio, full, 200.0, 150.0, khz, tail)


@pytest.mark.parametrize("ratio,full,tail", [(1.0, False, 0), (8.0, False, 0), (1.0, True, 0), (8.0, False, 1),
                                             (4.0, False, 2)])
def test_pipe_matches_oracle_elt(elt_loop, ratio, full, tail):
    sc, frames, ref = elt_loop
    with _ctx_for(sc) as ctx:
        khz = rtc.rtc_wall_clock_khz(ctx)
        out = _pipe_run(ctx, frames, alloc_ratio=ratio, full_frame=full, frame_period_us=1000.0,
                        readout_us=1000.0, rows_per_packet=2, tail_rows=tail)
    print(f"pipe info {out['info']}", flush=True)
    check_parity(out, ref, sc.cfg.gain, sc.cfg.leak, what=f"elt pipe ratio={ratio} full={full} tail={tail}")
    _check_arrival_order(sc, out, ratio, full, 1000.0, 1000.0, khz, tail)


@pytest.mark.parametrize("n_pix,ratio,tail", [(7, 1.0, 0), (7, 4.0, 1), (20, 4.0, 0), (20, 1.0, 2)])
def test_pipe_odd_and_wide_tiles_match_oracle(n_pix, ratio, tail):
    # odd tile sides (rows starting on odd pixels, single-pixel words) and
    # tiles wider than 16 pixels (32 lanes per tile)
    rng = np.random.default_rng(70 + n_pix + tail)
    n_sub = 12
    mask = geometry.subaperture_mask(n_sub, 0.2)
    nv = int(mask.sum())
    H = n_sub * n_pix
    F, n_act, gain, T = 4, 90, 0.4, 60.0
    frames = rng.integers(90, 400, size=(F, H, H)).astype(np.uint16)
    dark = rng.uniform(95.0, 105.0, size=(H, H)).astype(np.float32)
    flat = rng.normal(1.0, 0.02, size=(H, H)).astype(np.float32)
    R = (rng.standard_normal((n_act, 2 * nv)) / 100).astype(np.float32)
    ref = {k: [] for k in ("counts", "slopes", "recon", "cmd")}
    c = np.zeros(n_act)
    for f in range(F):
        r = oracle.rtc_frame(frames[f], mask, n_pix, dark, flat, T, R.astype(np.float64), c, gain)
        c = r["cmd"]
        for k in ref:
            ref[k].append(r[k])
    ref = {k: np.array(v) for k, v in ref.items()}
    with rtc.rtc_init(mask, n_pix, n_act, gain=gain) as ctx:
        rtc.rtc_load_calib(ctx, dark, flat, T)
        rtc.rtc_load_cmat(ctx, R)
        out = _pipe_run(ctx, frames, alloc_ratio=ratio, tail_rows=tail, frame_period_us=300.0)
    assert out["info"]["n_tail"] == np.count_nonzero(np.nonzero(mask)[0] >= n_sub - tail)
    check_parity(out, ref, gain, 1.0, what=f"pipe n_pix {n_pix}")


@pytest.mark.parametrize("fmt", ["f16", "bf16", "fp8e4m3"])
def test_pipe_reduced_formats_match_dequantised_oracle(tiny_loop, fmt):
    from test_gpu_precision import _dequantised_ref
    sc, frames, ref = tiny_loop
    with _ctx_for(sc, cm_dtype=fmt) as ctx:
        out = _pipe_run(ctx, frames[:40], n_workers=7, alloc_ratio=2.0, frame_period_us=200.0,
                        readout_us=150.0, tail_rows=1)
        rtc.rtc_reset(ctx)
        per = _gpu_batch(ctx, frames[:40])
    dq_ref, _ = _dequantised_ref({k: v[:40] for k, v in ref.items()}, sc.control_matrix, fmt, sc.cfg.gain,
                                 sc.cfg.leak)
    check_parity(out, dq_ref, sc.cfg.gain, sc.cfg.leak, what=f"tiny pipe {fmt} vs dequantised oracle")
    assert np.array_equal(out["counts"], per["counts"]) and np.array_equal(out["slopes"], per["slopes"])


def test_pipe_continues_the_integrator_state_and_chunks_compose(tiny_loop):
    sc, frames, ref = tiny_loop
    kw = dict(n_workers=7, alloc_ratio=3.0, frame_period_us=200.0, readout_us=150.0)
    with _ctx_for(sc) as ctx:
        first = _gpu_batch(ctx, frames[:10])                 # per-launch frames, then the pipe
        c0 = rtc.rtc_get_state(ctx)
        a = _pipe_run(ctx, frames[10:25], **kw)
        b = _pipe_run(ctx, frames[25:40], **kw)
        rtc.rtc_set_state(ctx, c0)
        whole = _pipe_run(ctx, frames[10:40], **kw)
    assert np.array_equal(c0, first["cmd"][-1])
    assert np.array_equal(np.concatenate([a["cmd"], b["cmd"]]), whole["cmd"])
    check_parity(whole, {k: v[10:40] for k, v in ref.items()}, sc.cfg.gain, sc.cfg.leak, c0=c0,
                 what="tiny pipe after per-launch frames")


def test_pipe_errors(tiny_loop):
    sc, frames, ref = tiny_loop
    pix = _dev(frames[:2].reshape(2, -1))
    cmd = torch.empty(2 * sc.n_act, dtype=torch.float32, device="cuda:0")
    with _ctx_for(sc) as ctx:
        with pytest.raises(rtc.RtcError) as e:
            rtc.rtc_pipe_run(ctx, 2, pix, cmd)
        assert e.value.status == rtc.RTC_E_STATE
        for bad in (dict(alloc_ratio=0.5), dict(readout_us=300.0, frame_period_us=200.0), dict(n_workers=100000),
                    dict(rows_per_packet=0), dict(wait_limit_us=-1), dict(tail_rows=-1), dict(tail_rows=11)):
            with pytest.raises(rtc.RtcError) as e:
                rtc.rtc_pipe_setup(ctx, **bad)
            assert e.value.status == rtc.RTC_E_ARG, bad
        with pytest.raises(rtc.RtcError) as e:
            rtc.rtc_pipe_setup(ctx, n_workers=1)                      # 97 actuator rows for one worker
        assert e.value.status == rtc.RTC_E_UNSUPPORTED
        rtc.rtc_pipe_setup(ctx, n_workers=4)
        pix3 = _dev(frames[:3].reshape(3, -1))
        with pytest.raises(rtc.RtcError) as e:
            rtc.rtc_pipe_run(ctx, 2, pix3, cmd, frame_stride=ctx.frame_elems + 1)
        assert e.value.status == rtc.RTC_E_ARG
        rtc.rtc_load_cmat(ctx, sc.control_matrix)                      # a new matrix needs a new setup
        with pytest.raises(rtc.RtcError) as e:
            rtc.rtc_pipe_run(ctx, 2, pix, cmd)
        assert e.value.status == rtc.RTC_E_STATE
    sensors = [(np.ones((2, 2), np.uint8), 4), (np.ones((3, 3), np.uint8), 4)]
    with rtc.rtc_init_multi(sensors, 5) as mctx:
        rtc.rtc_load_cmat(mctx, np.zeros((5, mctx.n_slopes), np.float32))
        with pytest.raises(rtc.RtcError) as e:
            rtc.rtc_pipe_setup(mctx, n_workers=2)
        assert e.value.status == rtc.RTC_E_UNSUPPORTED


def test_expired_pipe_wait_is_reported_and_cleared(tiny_loop):
    # A 1 us wait limit makes the workers' own bounded waits for the first rows
    # give up (the camera starts 200 us later); every workgroup winds down.
    sc, frames, ref = tiny_loop
    with _ctx_for(sc) as ctx:
        rtc.rtc_pipe_setup(ctx, n_workers=4, frame_period_us=200.0, readout_us=150.0, wait_limit_us=1)
        pix = _dev(frames[:3].reshape(3, -1))
        cmd = torch.zeros(3 * sc.n_act, dtype=torch.float32, device="cuda:0")
        rtc.rtc_pipe_run(ctx, 3, pix, cmd)
        with pytest.raises(rtc.RtcError) as e:
            rtc.rtc_sync_check(ctx)
        assert e.value.status == rtc.RTC_E_DEVICE
        rtc.rtc_sync_check(ctx)                                        # cleared
        rtc.rtc_reset(ctx)
        out = _pipe_run(ctx, frames[:20], n_workers=4, frame_period_us=200.0, readout_us=150.0)
    check_parity(out, {k: v[:20] for k, v in ref.items()}, sc.cfg.gain, sc.cfg.leak, what="tiny pipe after abort")
