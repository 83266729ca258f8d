"""Graph replay of frame batches and the autotuner (GPU)."""
import numpy as np
import pytest

from _closedloop import oracle_closed_loop, oracle_closed_loop_multi
from _gpu_helpers import _ctx_for, _dev, _gpu_batch, check_parity
from aosim import ELT, TINY, Scenario
from aosim.multi import TINY_MULTI, MultiScenario

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
    return (sc,) + oracle_closed_loop(sc, 48)


def _buffers(ctx, F):
    z = lambda n, dt=torch.float32: torch.zeros(n, dtype=dt, device="cuda:0")
    return dict(cmd=z(F * ctx.n_act), slopes=z(F * ctx.n_slopes), recon=z(F * ctx.n_act),
                counts=z(F * ctx.n_valid, torch.int32))


def _host(buf):
    return {k: v.cpu().numpy().copy() for k, v in buf.items()}


def _replays_match_eager(make_ctx, sets, mode, reps=3):
    F = sets.shape[0]
    pix = _dev(sets.reshape(F, -1))
    with make_ctx() as eager:
        rtc.rtc_set_frame_mode(eager, mode)
        eb = _buffers(eager, F)
        want = []
        for _ in range(reps):
            rtc.rtc_frame_batch(eager, F, pix, eb["cmd"], eb["slopes"], eb["recon"], eb["counts"])
            torch.cuda.synchronize()
            want.append(_host(eb))
    with make_ctx() as ctx:
        rtc.rtc_set_frame_mode(ctx, mode)
        gb = _buffers(ctx, F)
        try:
            rtc.rtc_graph_capture(ctx, F, pix, gb["cmd"], gb["slopes"], gb["recon"], gb["counts"])
        except rtc.RtcError as err:
            assert err.status == rtc.RTC_E_UNSUPPORTED and mode == rtc.RTC_FRAMES_PERSISTENT, err
            return False
        torch.cuda.synchronize()
        assert np.all(gb["cmd"].cpu().numpy() == 0), "capture must not run the frames"
        other = torch.ones(1 << 20, device="cuda:0")
        for r in range(reps):
            rtc.rtc_graph_launch(ctx)
            torch.cuda.synchronize()
            got = _host(gb)
            for k in got:
                assert np.array_equal(got[k], want[r][k]), f"replay {r}: {k} differs from the eager batch"
            other.mul_(1.0001).sum().item()            # unrelated eager work between replays
            torch.cuda.synchronize()
    return True


@pytest.mark.parametrize("mode", [rtc.RTC_FRAMES_PER_LAUNCH, rtc.RTC_FRAMES_PERSISTENT])
def test_graph_replays_equal_eager_batches(tiny_loop, mode):
    sc, frames, _ = tiny_loop
    # gfx950's runtime records cooperative launches, so both modes must record
    assert _replays_match_eager(lambda: _ctx_for(sc), frames[:16], mode), f"mode {mode}: capture refused"


def test_graph_replays_of_several_sensors():
    sc = MultiScenario(TINY_MULTI)
    sets, _ = oracle_closed_loop_multi(sc, 12)

    def make():
        ctx = rtc.rtc_init_multi(sc.sensors, sc.n_act, gain=sc.cfg.gain, leak=sc.cfg.leak)
        rtc.rtc_load_calib_multi(ctx, sc.dark_set, sc.flat_set, sc.thresholds)
        rtc.rtc_load_cmat(ctx, sc.control_matrix)
        return ctx
    for mode in (rtc.RTC_FRAMES_PER_LAUNCH, rtc.RTC_FRAMES_PERSISTENT):
        assert _replays_match_eager(make, sets, mode, reps=2), f"mode {mode}: capture refused"


def test_graph_launch_without_capture_is_a_state_error(tiny_loop):
    sc, _, _ = tiny_loop
    with _ctx_for(sc) as ctx:
        with pytest.raises(rtc.RtcError) as ei:
            rtc.rtc_graph_launch(ctx)
        assert ei.value.status == rtc.RTC_E_STATE


@pytest.mark.parametrize("fmt", ["f32", "bf16"])
def test_autotune_keeps_the_fastest_and_restores_state(fmt):
    sc = Scenario(ELT)
    frames, ref = oracle_closed_loop(sc, 4)
    ring = np.stack([sc.frame(100 + i, sc.turbulence_slopes(100 + i)) for i in range(8)])
    pix = _dev(np.tile(ring.reshape(8, -1), (8, 1)))
    cmd = torch.empty(64 * sc.n_act, device="cuda:0")
    with _ctx_for(sc, cm_dtype=fmt) as ctx:
        state = np.linspace(-1, 1, sc.n_act).astype(np.float32)
        rtc.rtc_set_state(ctx, state)
        res = rtc.rtc_autotune(ctx, 64, pix, cmd)
        assert np.array_equal(rtc.rtc_get_state(ctx), state)
        ok = [r for r in res if r["us_per_frame"] > 0]
        assert len(res) >= (17 if fmt == "f32" else 14) and len(ok) >= len(res) - 2
        best = min(ok, key=lambda r: r["us_per_frame"])
        assert rtc.rtc_get_frame_mode(ctx) == best["frame_mode"]
        assert rtc.rtc_get_mvm_tuning(ctx) == best["tuning"]
        print(f"{fmt}: best {best}", flush=True)
        # the tuned context still computes the frame
        rtc.rtc_reset(ctx)
        F = frames.shape[0]
        p2 = _dev(frames.reshape(F, -1))
        out = {k: torch.empty(F * n, dtype=dt, device="cuda:0") for k, n, dt in
               (("cmd", sc.n_act, torch.float32), ("slopes", 2 * sc.n_valid, torch.float32),
                ("recon", sc.n_act, torch.float32), ("counts", sc.n_valid, torch.int32))}
        rtc.rtc_frame_batch(ctx, F, p2, out["cmd"], out["slopes"], out["recon"], out["counts"])
        torch.cuda.synchronize()
        gpu = {k: v.cpu().numpy().reshape(F, -1) for k, v in out.items()}
    if fmt == "f32":
        check_parity(gpu, ref, sc.cfg.gain, sc.cfg.leak, what="after autotune")
    else:
        assert np.array_equal(gpu["counts"], ref["counts"])
