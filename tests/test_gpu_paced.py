"""Host-paced persistent batches: frames released one by one through a host
word, completion seen through another (latency as defined in Section 3)."""
import numpy as np
import pytest

from _closedloop import oracle_closed_loop
from _gpu_helpers import _ctx_for, _dev, check_parity
from aosim import ELT, TINY, Scenario

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
    return (sc,) + oracle_closed_loop(sc, 60)


@pytest.fixture(scope="module")
def elt_loop():
    sc = Scenario(ELT)
    return (sc,) + oracle_closed_loop(sc, 8)


def _outs(ctx, F):
    z = lambda n, dt=torch.float32: torch.zeros(n, dtype=dt, device="cuda:0")
    return dict(cmd=z(F * ctx.n_act), slopes=z(F * ctx.n_slopes), recon=z(F * ctx.n_act),
                counts=z(F * ctx.n_valid, torch.int32), ts=z(2 * F, torch.int64))


def _host(o, F):
    return {k: v.cpu().numpy().reshape(F, -1) for k, v in o.items()}


def _paced_vs_batch(sc, frames, period_us):
    F = frames.shape[0]
    pix = _dev(frames.reshape(F, -1))
    with _ctx_for(sc) as a, _ctx_for(sc) as b:
        for ctx in (a, b):
            rtc.rtc_set_frame_mode(ctx, rtc.RTC_FRAMES_PERSISTENT)
        oa, ob = _outs(a, F), _outs(b, F)
        print(f"paced batch: {F} frames every {period_us} us", flush=True)
        rel, done = rtc.rtc_paced_batch(a, F, pix, oa["cmd"], period_us, oa["slopes"], oa["recon"], oa["counts"],
                                        oa["ts"])
        rtc.rtc_frame_batch(b, F, pix, ob["cmd"], ob["slopes"], ob["recon"], ob["counts"], ob["ts"])
        torch.cuda.synchronize()
        rtc.rtc_sync_check(a)
        state_a, state_b = rtc.rtc_get_state(a), rtc.rtc_get_state(b)
        khz = rtc.rtc_wall_clock_khz(a)
    ga, gb = _host(oa, F), _host(ob, F)
    for key in ("counts", "slopes", "recon", "cmd"):
        assert np.array_equal(ga[key], gb[key]), key
    assert np.array_equal(state_a, state_b)
    # release k at t0 + k period or later; completion after release, in order
    assert np.all(rel >= np.arange(F) * period_us * 1e3)
    assert np.all(done > rel) and np.all(np.diff(done) > 0)
    starts_us = (ga["ts"][:, 0].astype(np.int64) - int(ga["ts"][0, 0])) * 1e3 / khz
    assert np.all(np.diff(starts_us) > 0)
    # the frames were held back: device starts span the release schedule
    assert starts_us[-1] >= 0.95 * (F - 1) * period_us, (starts_us[-1], F, period_us)
    return ga, rel, done


def test_paced_tiny_frames_equal_the_batch_and_the_oracle(tiny_loop):
    sc, frames, ref = tiny_loop
    ga, rel, done = _paced_vs_batch(sc, frames, 200.0)
    check_parity(ga, ref, sc.cfg.gain, sc.cfg.leak, what="tiny paced")
    print(f"host latency p50 {np.median(done - rel) / 1e3:.2f} us", flush=True)


def test_paced_elt_frames_equal_the_batch_and_the_oracle(elt_loop):
    sc, frames, ref = elt_loop
    ga, rel, done = _paced_vs_batch(sc, frames, 1000.0)
    check_parity(ga, ref, sc.cfg.gain, sc.cfg.leak, what="ELT paced")


def test_paced_batches_continue_from_state(tiny_loop):
    sc, frames, _ = tiny_loop
    F = 30
    pix = _dev(frames[:F].reshape(F, -1))
    with _ctx_for(sc) as a, _ctx_for(sc) as b:
        for ctx in (a, b):
            rtc.rtc_set_frame_mode(ctx, rtc.RTC_FRAMES_PERSISTENT)
        ca = torch.zeros(F * a.n_act, device="cuda:0")
        cb = torch.zeros(F * b.n_act, device="cuda:0")
        rtc.rtc_paced_batch(a, 10, pix, ca, 100.0)
        rtc.rtc_frame_batch(a, 10, pix[10:], ca[10 * a.n_act:])
        rtc.rtc_paced_batch(a, 10, pix[20:], ca[20 * a.n_act:], 100.0)
        rtc.rtc_frame_batch(b, F, pix, cb)
        torch.cuda.synchronize()
        rtc.rtc_sync_check(a)
        assert torch.equal(ca, cb)


def test_paced_batch_errors(tiny_loop):
    sc, frames, _ = tiny_loop
    pix = _dev(frames[:2].reshape(2, -1))
    with _ctx_for(sc) as ctx:
        cmd = torch.zeros(2 * ctx.n_act, device="cuda:0")
        with pytest.raises(rtc.RtcError) as ei:
            rtc.rtc_paced_batch(ctx, 2, pix, cmd, 100.0)      # per-launch mode
        assert ei.value.status == rtc.RTC_E_STATE
        rtc.rtc_set_frame_mode(ctx, rtc.RTC_FRAMES_PERSISTENT)
        for bad in (0.0, -5.0, 2e7):
            with pytest.raises(rtc.RtcError) as ei:
                rtc.rtc_paced_batch(ctx, 2, pix, cmd, bad)
            assert ei.value.status == rtc.RTC_E_ARG


def test_paced_batch_whose_device_wait_expires_fails_and_is_reported(tiny_loop):
    # A spin limit of one poll makes workgroup 0's wait for the first release
    # give up before the host releases it: the kernel winds down normally, the
    # host's wait for that frame times out, and the expired wait is reported.
    sc, frames, _ = tiny_loop
    pix = _dev(frames[:4].reshape(4, -1))
    with _ctx_for(sc) as ctx:
        rtc.rtc_set_frame_mode(ctx, rtc.RTC_FRAMES_PERSISTENT, spin_limit=1)
        cmd = torch.zeros(4 * ctx.n_act, device="cuda:0")
        with pytest.raises(rtc.RtcError) as ei:
            rtc.rtc_paced_batch(ctx, 4, pix, cmd, 1000.0)
        assert ei.value.status == rtc.RTC_E_DEVICE and "not done" in str(ei.value)
        with pytest.raises(rtc.RtcError) as ei:
            rtc.rtc_sync_check(ctx)
        assert ei.value.status == rtc.RTC_E_DEVICE
        rtc.rtc_reset(ctx)
        rtc.rtc_set_frame_mode(ctx, rtc.RTC_FRAMES_PERSISTENT)
        rel, done = rtc.rtc_paced_batch(ctx, 4, pix, cmd, 200.0)   # usable again
        assert np.all(done > rel)
