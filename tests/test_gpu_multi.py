"""Several wavefront sensors of uneven size reconstructed by one matrix (GPU).

The tiny multi-sensor loop (two 10x10 / 8 px sensors and one 4x4 / 6 px
sensor, 134 actuators on two DMs) is closed by the oracle and replayed on the
device; the ELT-size case (six 74x74 / 10 px and three 16x16 / 6 px sensors,
48,816 slopes, 4998 actuators, BF16 matrix) runs the full shape in both frame
modes against the float64 product with the dequantised matrix.
"""
import numpy as np
import pytest

import oracle
from _closedloop import oracle_closed_loop_multi
from _gpu_helpers import _gpu_batch, check_parity
from aosim.multi import ELT_MULTI, TINY_MULTI, MultiScenario
from oracle import quant

torch = pytest.importorskip("torch")
from paper_1805_07254_amd import rtc  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rtc.load_library()


@pytest.fixture(scope="module")
def tiny_multi():
    sc = MultiScenario(TINY_MULTI)
    sets, ref = oracle_closed_loop_multi(sc, 200)
    return sc, sets, ref


def _ctx(sc, fmt="f32", mode=rtc.RTC_FRAMES_PER_LAUNCH, R=None):
    cfg = sc.cfg
    ctx = rtc.rtc_init_multi(sc.sensors, sc.n_act, cm_dtype=fmt, gain=cfg.gain, leak=cfg.leak)
    rtc.rtc_load_calib_multi(ctx, sc.dark_set, sc.flat_set, sc.thresholds)
    rtc.rtc_load_cmat(ctx, sc.control_matrix if R is None else R)
    rtc.rtc_set_frame_mode(ctx, mode)
    return ctx


@pytest.mark.parametrize("mode", [rtc.RTC_FRAMES_PER_LAUNCH, rtc.RTC_FRAMES_PERSISTENT])
def test_tiny_multi_closed_loop_matches_oracle(tiny_multi, mode):
    sc, sets, ref = tiny_multi
    with _ctx(sc, mode=mode) as ctx:
        assert ctx.frame_elems == sets.shape[1] and ctx.n_slopes == 344
        gpu = _gpu_batch(ctx, sets)
        rtc.rtc_sync_check(ctx)
    check_parity(gpu, ref, sc.cfg.gain, sc.cfg.leak, what=f"tiny multi mode {mode}")


@pytest.mark.parametrize("fmt", ["f32", "f16", "bf16", "fp8e4m3"])
def test_tiny_multi_persistent_is_bitwise_per_launch(tiny_multi, fmt):
    sc, sets, _ = tiny_multi
    out = []
    for mode in (rtc.RTC_FRAMES_PER_LAUNCH, rtc.RTC_FRAMES_PERSISTENT):
        with _ctx(sc, fmt, mode) as ctx:
            out.append(_gpu_batch(ctx, sets[:40]))
            rtc.rtc_sync_check(ctx)
    for key in out[0]:
        assert np.array_equal(out[0][key], out[1][key]), key


def test_per_sensor_thresholds_apply_to_their_own_sensor(tiny_multi):
    sc, sets, _ = tiny_multi
    thr = [3.0, 40.0, 0.0]
    ref = [oracle.rtc_frame_multi(
        [sets[k][:6400].reshape(80, 80), sets[k][6400:12800].reshape(80, 80), sets[k][12800:].reshape(24, 24)],
        sc.sensors, sc.darks, sc.flats, thr, sc.control_matrix, np.zeros(sc.n_act), sc.cfg.gain) for k in range(3)]
    with _ctx(sc) as ctx:
        rtc.rtc_load_calib_multi(ctx, sc.dark_set, sc.flat_set, thr)
        for k in range(3):
            rtc.rtc_reset(ctx)
            gpu = _gpu_batch(ctx, sets[k:k + 1])
            assert np.array_equal(gpu["counts"][0], ref[k]["counts"])
            assert np.abs(gpu["slopes"][0] - ref[k]["slopes"]).max() <= 1e-5 * max(np.abs(ref[k]["slopes"]).max(), 0.1)


@pytest.fixture(scope="module")
def elt_multi_inputs():
    # full ELT multi-sensor shape; parity does not depend on how R was made, so a
    # seeded dense matrix of the Tikhonov matrix's magnitude stands in for it
    sc = MultiScenario(ELT_MULTI)
    rng = np.random.default_rng(3_180_507)
    R = (rng.standard_normal((sc.n_act, sc.n_slopes), dtype=np.float32) * np.float32(0.02))
    sets = []
    for k in range(3):
        s = rng.standard_normal(sc.n_slopes) * 0.8
        sets.append(sc.frame_set(k, s))
    return sc, R, np.stack(sets)


@pytest.mark.parametrize("fmt", ["bf16", "f16", "fp8e4m3"])
def test_elt_multi_full_shape_both_modes(elt_multi_inputs, fmt):
    # every format runs in slope panels at this slope count (FP8 from 4 chunks
    # per lane on, BF16 and F16 from 8)
    sc, R, sets = elt_multi_inputs
    out = []
    for mode in (rtc.RTC_FRAMES_PER_LAUNCH, rtc.RTC_FRAMES_PERSISTENT):
        with _ctx(sc, fmt, mode, R=R) as ctx:
            out.append(_gpu_batch(ctx, sets))
            rtc.rtc_sync_check(ctx)
    for key in out[0]:
        assert np.array_equal(out[0][key], out[1][key]), key
    # the oracle's own frames with the dequantised matrix: counts, slopes,
    # reconstruction and the integrator, frame by frame
    Rq = quant.dequantize(*quant.encode(R, fmt), fmt)
    c = np.zeros(sc.n_act)
    frames_of = lambda k: [sets[k][o:o + h * h].reshape(h, h) for o, h in _offsets(sc)]
    refs = []
    for k in range(3):
        ref = oracle.rtc_frame_multi(frames_of(k), sc.sensors, sc.darks, sc.flats, sc.thresholds, Rq, c,
                                     sc.cfg.gain, sc.cfg.leak)
        c = ref["cmd"]
        refs.append(ref)
        a_gpu = out[0]["slopes"][k].astype(np.float64) @ Rq.T     # same slopes: accumulation only
        assert np.abs(out[0]["recon"][k] - a_gpu).max() <= 1e-5 * np.abs(a_gpu).max()
    ref = {key: np.stack([r[key] for r in refs]) for key in ("counts", "slopes", "recon", "cmd")}
    gpu = {key: out[0][key][:3] for key in ("counts", "slopes", "recon", "cmd")}
    check_parity(gpu, ref, sc.cfg.gain, sc.cfg.leak, what=f"ELT multi-sensor {fmt}")


def _offsets(sc):
    o, out = 0, []
    for w in range(len(sc.cfg.sensors)):
        h = sc.frame_side(w)
        out.append((o, h))
        o += h * h
    return out
