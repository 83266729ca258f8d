"""What the learned predictor gains over the plain integrator (GPU).

Tiny SCAO geometry (10x10 subapertures, 97 actuators) under two frozen-flow
layers (8 and 20 m/s at 1 kHz) with 0.05 px slope noise.  The integrator's
closed loop generates the telemetry (disjoint training, validation and test
seeds); the change of 40 pseudo-open-loop KL modes is forecast from the last
5 frames by a 200 -> 256 -> 40 network trained with the library's kernels and
fed forward into the same integrator; on the test segment the residual slope
RMS must be lower than the plain integrator's (gain 0.4), which is the judge.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from aosim import TINY, Scenario  # noqa: E402
from aosim.telemetry import Telemetry, kl_basis  # noqa: E402
from paper_1805_07254_amd import predict, rtc  # noqa: E402

pytestmark = pytest.mark.gpu

N_MODES, HISTORY, HIDDEN, SEG, N_TRAIN = 40, 5, 256, 2000, 10


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rtc.load_library()


def test_trained_predictor_beats_the_integrator():
    sc = Scenario(TINY)
    dev = torch.device("cuda:0")
    D = torch.from_numpy(sc.interaction.astype(np.float32)).to(dev)
    R = sc.control_matrix
    tel = Telemetry(sc.mask, sc.cfg.pitch, config_index=0, device=dev)
    ns = 2 * sc.n_valid
    ctx = predict.make_context(sc, R, gain=sc.cfg.gain)

    # closed-loop telemetry of the plain integrator
    res, cprev, ol = [], [], []
    for seg in range(N_TRAIN + 1):
        s = tel.segment(seg, SEG)
        out = predict.run_loop(D, s, tel.noise(seg, SEG, ns), ctx)
        res.append(out["residual"])
        cprev.append(out["cmd_prev"])
        ol.append(s[::10])
    # training-set preparation on the host (offline work)
    P = kl_basis(torch.cat(ol[:N_TRAIN]), N_MODES)
    PD = (P.astype(np.float64) @ sc.interaction.astype(np.float64)).astype(np.float32)
    m_all = [predict.pol_modes(r, c, P, PD) for r, c in zip(res, cprev)]
    mean, std = predict.change_stats(np.concatenate(m_all[:N_TRAIN]))
    xs, ys = zip(*[predict.windows(m, HISTORY, mean, std) for m in m_all[:N_TRAIN]])
    x, y = predict.to_device(np.concatenate(xs), dev), predict.to_device(np.concatenate(ys), dev)
    xv_h, yv_h = predict.windows(m_all[N_TRAIN], HISTORY, mean, std)
    xv, yv = predict.to_device(xv_h, dev), predict.to_device(yv_h, dev)

    net = rtc.MlpNet(HISTORY * N_MODES, HIDDEN, N_MODES, 256)
    net.set_params(*predict.init_params(HISTORY * N_MODES, HIDDEN, N_MODES, seed=5))
    before = predict.evaluate(net, xv, yv, 256)
    persist = float(((xv_h[:, -N_MODES:].astype(np.float64) - yv_h) ** 2).mean())   # forecast = the last change again
    hist = predict.train(net, x, y, epochs=8, batch=256, lr=2e-3, seed=6, x_val=xv, y_val=yv)
    after = hist[-1]["val_loss"]
    print(f"validation MSE (normalised changes): untrained {before:.4f}, last change {persist:.4f}, "
          f"trained {after:.4f}", flush=True)
    # the network starts near "no change" (small output layer); training must beat
    # both that and repeating the last change
    assert after < before and after < 0.9 * persist

    # judge on a held-out segment
    seg = N_TRAIN + 1
    s = tel.segment(seg, SEG)
    nz = tel.noise(seg, SEG, ns)
    base = predict.run_loop(D, s, nz, ctx)
    pred = rtc.Predictor(net, HISTORY, P, PD, mean, std, sc.cfg.gain)
    out = predict.run_loop(D, s, nz, ctx, pred)
    r_int = predict.residual_rms(base["residual"], 100)
    r_pred = predict.residual_rms(out["residual"], 100)
    ol_rms = predict.residual_rms(s + nz, 100)
    print(f"residual slope RMS (px): open loop {ol_rms:.4f}, integrator {r_int:.4f}, predictive {r_pred:.4f} "
          f"({100 * (1 - r_pred / r_int):.1f} % lower)", flush=True)
    assert r_pred < r_int
    pred.close()
    net.close()
