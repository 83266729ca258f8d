"""The predictor's network on the device against the float64 oracle (GPU):
forward, gradients, Adam and the modal predictor step, with element-wise
bounds derived from float32 accumulation and bfloat16 rounding."""
import numpy as np
import pytest

from _mlp_bounds import U, forward_bounds, grad_bounds
from oracle import predictor as pr

torch = pytest.importorskip("torch")
from paper_1805_07254_amd import rtc  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rtc.load_library()


def _params(rng, n_in, n_hid, n_out, scale=1.0):
    return [(rng.standard_normal((n_hid, n_in)) * scale / np.sqrt(n_in)).astype(np.float32),
            (rng.standard_normal(n_hid) * 0.1).astype(np.float32),
            (rng.standard_normal((n_out, n_hid)) * scale / np.sqrt(n_hid)).astype(np.float32),
            (rng.standard_normal(n_out) * 0.1).astype(np.float32)]


def _d(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


SHAPES = [(5, 7, 3, 4), (40, 33, 17, 31), (130, 96, 65, 64), (2500, 1024, 500, 64)]


@pytest.mark.parametrize("n_in,n_hid,n_out,B", SHAPES)
def test_forward_matches_oracle(n_in, n_hid, n_out, B):
    rng = np.random.default_rng(n_in + B)
    params = _params(rng, n_in, n_hid, n_out)
    X = rng.standard_normal((B, n_in)).astype(np.float32)
    with rtc.MlpNet(n_in, n_hid, n_out, max(B, 8)) as net:
        net.set_params(*params)
        y = torch.empty(B * n_out, device="cuda:0")
        net.forward(B, _d(X), y)
        torch.cuda.synchronize()
        got = y.cpu().numpy().reshape(B, n_out).astype(np.float64)
    f, e = forward_bounds(params, X)
    err = np.abs(got - f["Y"])
    assert np.all(err <= e["Y"]), f"max excess {np.max(err - e['Y'])}, worst err {err.max()}"
    print(f"forward {n_in}x{n_hid}x{n_out} B={B}: max err {err.max():.3e}, max bound {e['Y'].max():.3e}, "
          f"bf16 flips possible in H: {int(np.count_nonzero(e['Hr']))}", flush=True)


@pytest.mark.parametrize("n_in,n_hid,n_out,B", SHAPES)
def test_gradients_match_oracle(n_in, n_hid, n_out, B):
    rng = np.random.default_rng(100 + n_in + B)
    params = _params(rng, n_in, n_hid, n_out)
    X = rng.standard_normal((B, n_in)).astype(np.float32)
    T = rng.standard_normal((B, n_out)).astype(np.float32)
    with rtc.MlpNet(n_in, n_hid, n_out, B) as net:
        net.set_params(*params)
        loss = torch.zeros(1, device="cuda:0")
        net.loss_grad(B, _d(X), _d(T), loss)
        got = net.get_grads()
        got_loss = float(loss.item())
    ref_loss, ref, bounds, eloss, _ = grad_bounds(params, X, T)
    assert abs(got_loss - ref_loss) <= eloss
    for name, g, r, b in zip(("dW1", "db1", "dW2", "db2"), got, ref, bounds):
        err = np.abs(g.astype(np.float64) - r)
        assert np.all(err <= b), f"{name}: max excess {np.max(err - b)}, worst err {err.max()}, scale {np.abs(r).max()}"


def test_adam_steps_match_oracle():
    # W1 = b1 = W2 = 0 gives H = GELU(0) = 0 exactly, so at every step the
    # gradients of W1, b1 and W2 are exactly zero and that of b2 is an exact
    # dyadic sum: the optimiser itself is compared over several steps
    rng = np.random.default_rng(7)
    n_in, n_hid, n_out, B = 24, 16, 8, 16
    params = [np.zeros((n_hid, n_in), np.float32), np.zeros(n_hid, np.float32),
              np.zeros((n_out, n_hid), np.float32), (rng.integers(-8, 8, n_out) / 8.0).astype(np.float32)]
    X = rng.standard_normal((B, n_in)).astype(np.float32)
    T = (rng.integers(-16, 16, (B, n_out)) / 16.0).astype(np.float32)
    with rtc.MlpNet(n_in, n_hid, n_out, B) as net:
        net.set_params(*params)
        loss = torch.zeros(1, device="cuda:0")
        th, m, v = params[3].astype(np.float64), np.zeros(n_out), np.zeros(n_out)
        for step in range(1, 6):
            cur = params[:3] + [th.astype(np.float32)]
            net.loss_grad(B, _d(X), _d(T), loss)
            got = net.get_grads()
            _, grads, _ = pr.loss_grad(cur, X, T)
            assert all(np.all(g == 0) for g in got[:3]) and all(np.all(g == 0) for g in grads[:3])
            # db2 is exact on both sides only if b2 stays dyadic; compare within float32 rounding
            assert np.allclose(got[3], grads[3], rtol=2.0 ** -20, atol=0)
            net.adam(1e-2, step, 0.9, 0.999, 1e-8)
            th, m, v = pr.adam(th, m, v, grads[3], 1e-2, 0.9, 0.999, 1e-8, step)
            W1, b1, W2, b2 = net.get_params()
            assert not W1.any() and not b1.any() and not W2.any()
            assert np.allclose(b2, th, rtol=0, atol=8 * 2.0 ** -24 * np.abs(th).max()), step
        assert not np.array_equal(b2, params[3])


def test_predictor_step_matches_oracle():
    rng = np.random.default_rng(11)
    nm, ns, na, hist, hid, gain = 20, 200, 100, 3, 64, 0.4
    P = np.linalg.qr(rng.standard_normal((ns, nm)))[0].T.astype(np.float32)
    PD = (rng.standard_normal((nm, na)) / np.sqrt(na)).astype(np.float32)
    mean = (rng.standard_normal(nm) * 0.1).astype(np.float32)
    std = (0.5 + rng.random(nm)).astype(np.float32)
    params = _params(rng, hist * nm, hid, nm, 0.5)
    with rtc.MlpNet(hist * nm, hid, nm, 4) as net:
        net.set_params(*params)
        pred = rtc.Predictor(net, hist, P, PD, mean, std, gain)
        state = {}
        m_prev_err = None
        r_out = torch.empty(ns, device="cuda:0")
        modes = torch.empty(2 * nm, device="cuda:0")
        for k in range(7):
            r = rng.standard_normal(ns).astype(np.float32)
            c_prev = (rng.standard_normal(na) * 0.3).astype(np.float32)
            pred.step(_d(r), _d(c_prev), r_out, modes)
            torch.cuda.synchronize()
            r_ref, m_ref, mhat_ref, state = pr.predictor_step(params, state, r, c_prev, P, PD, mean, std, hist,
                                                              gain)
            window = state["window"]
            got_m = modes.cpu().numpy()[:nm].astype(np.float64)
            got_mhat = modes.cpu().numpy()[nm:].astype(np.float64)
            em = 1.5 * (ns + na) * U * (np.abs(P) @ np.abs(r) + np.abs(PD) @ np.abs(c_prev)) + U * np.abs(m_ref)
            assert np.all(np.abs(got_m - m_ref) <= em)
            em_max = em if m_prev_err is None else np.maximum(em, m_prev_err)
            m_prev_err = em
            d_ref = mhat_ref - m_ref
            if len(window) < hist:
                ed = np.zeros(nm)
            else:                                            # network on the normalised changes
                X = np.concatenate(window)[None, :]
                # a change carries the errors of two projections; earlier frames' errors are
                # bounded by the largest seen (inputs of the same scale)
                eX = np.concatenate([2 * em_max / std] * hist)[None, :] * 2 + 4 * U * np.abs(X)
                f, e = forward_bounds(params, X, eX)
                ed = e["Y"][0] * std + 2 * U * np.abs(d_ref)
            assert np.all(np.abs(got_mhat - mhat_ref) <= em + ed + U * np.abs(mhat_ref)), k
            er = (1.5 * nm * U * (np.abs(P.T) @ np.abs(d_ref)) + np.abs(P.T) @ ed) / gain + 2 * U * np.abs(r_ref)
            assert np.all(np.abs(r_out.cpu().numpy() - r_ref) <= er + 1e-30), k
        pred.close()
