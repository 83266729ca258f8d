"""Predictive frames (rtc_pred_frame_batch): the per-launch frame with the
predictor step between the slopes and the reconstruction, against the same
steps called one by one and, before the network's window fills, against the
plain integrator."""
import numpy as np
import pytest

from _gpu_helpers import _ctx_for, _dev
from aosim import TINY, Scenario

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

