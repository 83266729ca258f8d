"""Predictive frames (rtc_pred_frame_batch): the per-launch frame with the
predictor step between the slopes and the reconstruction, against the same
steps called one by one and, before the network's window fills, against the
plain integrator; the persistent form (one launch, the step's phases between
grid barriers) against the per-launch form, bit for bit, at the tiny and the
ELT shape."""
import numpy as np
import pytest

from _gpu_helpers import _ctx_for, _dev
from aosim import ELT, TINY, Scenario

torch = pytest.importorskip("torch")
from paper_1805_07254_amd import rtc  # noqa: E402

pytestmark = pytest.mark.gpu

NM, HIST, HID = 12, 3, 48


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rtc.load_library()


@pytest.fixture(scope="module")
def setup():
    sc = Scenario(TINY)
    F = 16
    frames = np.stack([sc.frame(i, sc.turbulence_slopes(i)) for i in range(F)])
    rng = np.random.default_rng(5)
    ns, na = 2 * sc.n_valid, sc.n_act
    P = np.linalg.qr(rng.standard_normal((ns, NM)))[0].T.astype(np.float32)
    PD = (rng.standard_normal((NM, na)) / np.sqrt(na)).astype(np.float32)
    mean = (rng.standard_normal(NM) * 0.01).astype(np.float32)
    std = (0.05 + 0.1 * rng.random(NM)).astype(np.float32)
    params = [(rng.standard_normal((HID, HIST * NM)) * 0.3 / np.sqrt(HIST * NM)).astype(np.float32),
              (rng.standard_normal(HID) * 0.1).astype(np.float32),
              (rng.standard_normal((NM, HID)) * 0.3 / np.sqrt(HID)).astype(np.float32),
              (rng.standard_normal(NM) * 0.1).astype(np.float32)]
    return sc, frames, (P, PD, mean, std, params)


def _predictor(net, sc, model):
    P, PD, mean, std, params = model
    net.set_params(*params)
    return rtc.Predictor(net, HIST, P, PD, mean, std, sc.cfg.gain)


def test_predictive_frames_equal_the_steps_called_one_by_one(setup):
    sc, frames, model = setup
    F = frames.shape[0]
    pix = _dev(frames.reshape(F, -1))
    with rtc.MlpNet(HIST * NM, HID, NM, 4) as na_, rtc.MlpNet(HIST * NM, HID, NM, 4) as nb_, \
            _ctx_for(sc) as a, _ctx_for(sc) as b:
        pa, pb = _predictor(na_, sc, model), _predictor(nb_, sc, model)
        cmd_a = torch.zeros(F * a.n_act, device="cuda:0")
        s_a = torch.zeros(F * a.n_slopes, device="cuda:0")
        ts = torch.zeros(2 * F, dtype=torch.int64, device="cuda:0")
        print(f"predictive batch of {F} tiny frames", flush=True)
        pa.frame_batch(a, F, pix, cmd_a, s_a, ts)
        cmd_b = torch.zeros(F * b.n_act, device="cuda:0")
        s_b = torch.zeros(F * b.n_slopes, device="cuda:0")
        s_out = torch.zeros(b.n_slopes, device="cuda:0")
        c_prev = torch.zeros(b.n_act, device="cuda:0")
        for k in range(F):
            rtc.rtc_calibrate_centroid(b, pix[k], s_b[k * b.n_slopes:(k + 1) * b.n_slopes])
            pb.step(s_b[k * b.n_slopes:(k + 1) * b.n_slopes], c_prev, s_out)
            rtc.rtc_reconstruct_integrate(b, s_out, cmd_b[k * b.n_act:(k + 1) * b.n_act])
            c_prev.copy_(cmd_b[k * b.n_act:(k + 1) * b.n_act])
        torch.cuda.synchronize()
        assert torch.equal(s_a, s_b)
        assert torch.equal(cmd_a, cmd_b)
        assert np.array_equal(rtc.rtc_get_state(a), rtc.rtc_get_state(b))
        t = ts.cpu().numpy().reshape(F, 2)
        assert np.all(t[:, 1] > t[:, 0]) and np.all(np.diff(t[:, 0]) > 0)
        pa.close()
        pb.close()


def test_predictive_frames_are_the_integrator_until_the_window_fills(setup):
    # the first HIST frames carry no forecast (d = 0), so r' = r exactly
    sc, frames, model = setup
    F = HIST
    pix = _dev(frames[:F].reshape(F, -1))
    with rtc.MlpNet(HIST * NM, HID, NM, 4) as net, _ctx_for(sc) as a, _ctx_for(sc) as b:
        p = _predictor(net, sc, model)
        cmd_a = torch.zeros(F * a.n_act, device="cuda:0")
        cmd_b = torch.zeros(F * b.n_act, device="cuda:0")
        p.frame_batch(a, F, pix, cmd_a)
        rtc.rtc_frame_batch(b, F, pix, cmd_b)
        torch.cuda.synchronize()
        assert torch.equal(cmd_a, cmd_b)
        p.close()



def _model(sc, nm, hist, hid, seed):
    rng = np.random.default_rng(seed)
    ns, na = 2 * sc.n_valid, sc.n_act
    P = np.linalg.qr(rng.standard_normal((ns, nm)))[0].T.astype(np.float32)
    PD = (rng.standard_normal((nm, na)) / np.sqrt(na)).astype(np.float32)
    mean = (rng.standard_normal(nm) * 0.01).astype(np.float32)
    std = (0.05 + 0.1 * rng.random(nm)).astype(np.float32)
    params = [(rng.standard_normal((hid, hist * nm)) * 0.3 / np.sqrt(hist * nm)).astype(np.float32),
              (rng.standard_normal(hid) * 0.1).astype(np.float32),
              (rng.standard_normal((nm, hid)) * 0.3 / np.sqrt(hid)).astype(np.float32),
              (rng.standard_normal(nm) * 0.1).astype(np.float32)]
    return P, PD, mean, std, params


def _persistent_vs_per_launch(sc, frames, nm, hist, hid, model, chunks, expect_mode):
    """Batches of the given sizes in both modes, one after another (the
    predictor and integrator state carried across batches), compared bit for
    bit after every batch."""
    F = frames.shape[0]
    assert sum(chunks) == F
    pix = _dev(frames.reshape(F, -1))
    P, PD, mean, std, params = model
    with rtc.MlpNet(hist * nm, hid, nm, 4) as na_, rtc.MlpNet(hist * nm, hid, nm, 4) as nb_, \
            _ctx_for(sc) as a, _ctx_for(sc) as b:
        rtc.rtc_set_frame_mode(a, rtc.RTC_FRAMES_PERSISTENT)
        na_.set_params(*params)
        nb_.set_params(*params)
        pa = rtc.Predictor(na_, hist, P, PD, mean, std, sc.cfg.gain)
        pb = rtc.Predictor(nb_, hist, P, PD, mean, std, sc.cfg.gain)
        z = lambda n, dt=torch.float32: torch.zeros(n, dtype=dt, device="cuda:0")  # noqa: E731
        cmd_a, cmd_b = z(F * a.n_act), z(F * b.n_act)
        s_a, s_b = z(F * a.n_slopes), z(F * b.n_slopes)
        ts_a = z(2 * F, torch.int64)
        f0 = 0
        for n in chunks:
            print(f"predictive batch of {n} frames from {f0}: persistent context, per-launch context", flush=True)
            pa.frame_batch(a, n, pix[f0:], cmd_a[f0 * a.n_act:], s_a[f0 * a.n_slopes:], ts_a[2 * f0:])
            assert pa.last_batch_mode() == expect_mode
            pb.frame_batch(b, n, pix[f0:], cmd_b[f0 * b.n_act:], s_b[f0 * b.n_slopes:])
            assert pb.last_batch_mode() == rtc.RTC_FRAMES_PER_LAUNCH
            torch.cuda.synchronize()
            rtc.rtc_sync_check(a)
            f1 = f0 + n
            assert torch.equal(s_a[:f1 * a.n_slopes], s_b[:f1 * b.n_slopes]), f"slopes, frames < {f1}"
            assert torch.equal(cmd_a[:f1 * a.n_act], cmd_b[:f1 * b.n_act]), f"commands, frames < {f1}"
            assert np.array_equal(rtc.rtc_get_state(a), rtc.rtc_get_state(b))
            f0 = f1
        t = ts_a.cpu().numpy().reshape(F, 2)
        assert np.all(t[:, 1] > t[:, 0]) and np.all(np.diff(t[:, 0]) > 0)
        # the forecast changed the commands once the window was full
        with _ctx_for(sc) as c:
            cmd_c = z(F * c.n_act)
            rtc.rtc_frame_batch(c, F, pix, cmd_c)
            torch.cuda.synchronize()
            assert not torch.equal(cmd_c, cmd_a)
        pa.close()
        pb.close()


def test_persistent_predictive_frames_equal_the_per_launch_ones(setup):
    sc, frames, _ = setup
    model = _model(sc, NM, HIST, HID, 11)
    # batches shorter than, equal to and longer than the window, so that the
    # ring and the frames seen carry over between launches at every stage
    _persistent_vs_per_launch(sc, frames, NM, HIST, HID, model, [2, 3, 11], rtc.RTC_FRAMES_PERSISTENT)


def test_predictive_frames_whose_network_is_not_built_persistent_run_per_launch(setup):
    # 13 modes x 3 frames = 39 inputs: the 8-byte weight rows the persistent
    # phases read need a multiple of 4, so the batch runs per launch
    sc, frames, _ = setup
    model = _model(sc, 13, HIST, HID, 12)
    _persistent_vs_per_launch(sc, frames[:6], 13, HIST, HID, model, [6], rtc.RTC_FRAMES_PER_LAUNCH)


@pytest.fixture(scope="module")
def elt_frames():
    sc = Scenario(ELT)
    F = 9
    frames = np.stack([sc.frame(i, sc.turbulence_slopes(i)) for i in range(F)])
    return sc, frames


def test_persistent_predictive_elt_frames_equal_the_per_launch_ones(elt_frames):
    # the benchmark's predictor shape: 500 modes, 5 frames of history, 1024 hidden units
    sc, frames = elt_frames
    nm, hist, hid = 500, 5, 1024
    model = _model(sc, nm, hist, hid, 13)
    _persistent_vs_per_launch(sc, frames, nm, hist, hid, model, [4, 5], rtc.RTC_FRAMES_PERSISTENT)


def test_persistent_predictive_batch_whose_wait_expires_is_reported(setup):
    # A spin limit of one poll makes the kernel's own bounded waits (five per
    # predictive frame) give up: the batch winds down normally, the host is
    # told, and after both resets the frames equal the per-launch ones again.
    sc, frames, _ = setup
    F = frames.shape[0]
    P, PD, mean, std, params = _model(sc, NM, HIST, HID, 14)
    pix = _dev(frames.reshape(F, -1))
    with rtc.MlpNet(HIST * NM, HID, NM, 4) as na_, rtc.MlpNet(HIST * NM, HID, NM, 4) as nb_, \
            _ctx_for(sc) as a, _ctx_for(sc) as b:
        na_.set_params(*params)
        nb_.set_params(*params)
        pa = rtc.Predictor(na_, HIST, P, PD, mean, std, sc.cfg.gain)
        pb = rtc.Predictor(nb_, HIST, P, PD, mean, std, sc.cfg.gain)
        cmd_a = torch.zeros(F * a.n_act, device="cuda:0")
        cmd_b = torch.zeros(F * b.n_act, device="cuda:0")
        rtc.rtc_set_frame_mode(a, rtc.RTC_FRAMES_PERSISTENT, spin_limit=1)
        print("predictive persistent batch with a spin limit of one poll", flush=True)
        pa.frame_batch(a, F, pix, cmd_a)
        assert pa.last_batch_mode() == rtc.RTC_FRAMES_PERSISTENT
        torch.cuda.synchronize()
        with pytest.raises(rtc.RtcError) as ei:
            rtc.rtc_sync_check(a)
        assert ei.value.status == rtc.RTC_E_DEVICE
        rtc.rtc_reset(a)
        pa.reset()
        rtc.rtc_set_frame_mode(a, rtc.RTC_FRAMES_PERSISTENT)
        pa.frame_batch(a, F, pix, cmd_a)
        pb.frame_batch(b, F, pix, cmd_b)
        torch.cuda.synchronize()
        rtc.rtc_sync_check(a)
        assert torch.equal(cmd_a, cmd_b)
        pa.close()
        pb.close()
