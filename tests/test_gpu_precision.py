"""Reduced-precision control matrices on the GPU (binary16, bfloat16, FP8 E4M3).

(i) Parity: the HIP reconstruction with a stored matrix equals the oracle's
reconstruction with the *dequantised* matrix within the float32 gates (only the
accumulation differs).  (ii) Against the float64 oracle with the unquantised
matrix, every actuator's error stays within the rigorous per-row bound
sum_j |R~_rj - R_rj| |s_j| plus float32 accumulation, and the RMS error of
the DM-command update is reported per format.
"""
import numpy as np
import pytest

import oracle
from _closedloop import oracle_closed_loop
from _gpu_helpers import TOL, _dev, _gpu_batch, check_parity, dequantised_ref
from aosim import ELT, TINY, Scenario
from oracle import quant

torch = pytest.importorskip("torch")
from paper_1805_07254_amd import rtc  # noqa: E402

pytestmark = pytest.mark.gpu
FMTS = ["f16", "bf16", "fp8e4m3"]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rtc.load_library()


@pytest.mark.parametrize("fmt", FMTS)
def test_every_code_decodes_exactly_on_the_device(fmt):
    # row r = [2^E, v_r]: the row scale is 1 and v_r is stored as its own code, so
    # the reconstruction with slopes (0, 1) returns exactly the decoded value.
    ebits, fbits, bias, E, _ = quant.FORMATS[fmt]
    nb = 1 + ebits + fbits
    codes = np.arange(1 << nb)
    vals = quant.decode_codes(codes, fmt)
    exp_field = (codes >> fbits) & ((1 << ebits) - 1)
    finite = (codes & 0x7F) != 0x7F if fmt == "fp8e4m3" else exp_field != (1 << ebits) - 1
    keep = finite & (np.abs(vals) <= 2.0 ** E)
    v = vals[keep]
    R = np.stack([np.full(len(v), 2.0 ** E), v], axis=1).astype(np.float32)
    c_codes, c_scales = quant.encode(R, fmt)
    assert np.all(c_scales == 1.0) and np.array_equal(c_codes[:, 1], codes[keep].astype(c_codes.dtype))
    n = len(v)
    with rtc.rtc_init(np.ones((1, 1), np.uint8), 2, n, cm_dtype=fmt, gain=1.0, leak=0.0) as ctx:
        rtc.rtc_load_calib(ctx, np.zeros((2, 2), np.float32), np.ones((2, 2), np.float32), 0.0)
        rtc.rtc_load_cmat(ctx, R)
        s = _dev(np.array([0.0, 1.0], np.float32))
        cmd = torch.empty(n, dtype=torch.float32, device="cuda:0")
        rec = torch.empty(n, dtype=torch.float32, device="cuda:0")
        rtc.rtc_reconstruct_integrate(ctx, s, cmd, rec)
        torch.cuda.synchronize()
        got = rec.cpu().numpy().astype(np.float64)
    bad = np.nonzero(got != v)[0]
    assert len(bad) == 0, f"{fmt}: {len(bad)} codes decode differently, e.g. code " \
                          f"{codes[keep][bad[:4]]} -> {got[bad[:4]]} instead of {v[bad[:4]]}"


def _dequantised_ref(ref, R, fmt, gain, leak):
    return dequantised_ref(ref, R, fmt, gain, leak)


def _check_error_bound(gpu_recon, ref, R, Rq, fmt):
    """Per-row rigorous bound against the unquantised float64 reconstruction; returns RMS rel error."""
    R64 = R.astype(np.float64)
    rms = []
    for k in range(gpu_recon.shape[0]):
        s = ref["slopes"][k]
        exact = R64 @ s
        bound = np.abs(Rq - R64) @ np.abs(s) + TOL * np.abs(Rq @ s).max()
        err = np.abs(gpu_recon[k].astype(np.float64) - exact)
        assert np.all(err <= bound), f"{fmt} frame {k}: error exceeds the quantisation bound"
        rms.append(np.sqrt(np.mean((gpu_recon[k] - exact) ** 2) / np.mean(exact ** 2)))
    return float(np.max(rms))


@pytest.fixture(scope="module")
def tiny_loop():
    sc = Scenario(TINY)
    frames, ref = oracle_closed_loop(sc, 200)
    return sc, frames, ref


@pytest.fixture(scope="module")
def elt_loop():
    sc = Scenario(ELT)
    frames, ref = oracle_closed_loop(sc, 4)
    return sc, frames, ref


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("which", ["tiny", "elt"])
def test_reduced_precision_replay(fmt, which, request):
    sc, frames, ref = request.getfixturevalue(f"{which}_loop")
    cfg = sc.cfg
    R = sc.control_matrix
    with rtc.rtc_init(sc.mask, cfg.n_pix, sc.n_act, cm_dtype=fmt, gain=cfg.gain, leak=cfg.leak) as ctx:
        rtc.rtc_load_calib(ctx, sc.dark, sc.flat, cfg.threshold)
        rtc.rtc_load_cmat(ctx, R)
        gpu = _gpu_batch(ctx, frames)
        rtc.rtc_reset(ctx)
        gpu16 = _gpu_batch(ctx, frames[:2], tuning=dict(waves=16, rows_per_wave=1))
    dq_ref, Rq = _dequantised_ref(ref, R, fmt, cfg.gain, cfg.leak)
    check_parity(gpu, dq_ref, cfg.gain, cfg.leak, what=f"{which} {fmt} vs dequantised oracle")
    check_parity(gpu16, {k: v[:2] for k, v in dq_ref.items()}, cfg.gain, cfg.leak, what=f"{which} {fmt} W16")
    rel = _check_error_bound(gpu["recon"], ref, R, Rq, fmt)
    print(f"{which} {fmt}: max per-frame RMS relative error of a = R s vs float64 unquantised: {rel:.3e}",
          flush=True)
    assert rel < {"f16": 2e-3, "bf16": 1e-2, "fp8e4m3": 8e-2}[fmt]


def test_streamed_kernel_reads_float32_only():
    with rtc.rtc_init(np.ones((2, 2), np.uint8), 2, 3, cm_dtype="bf16") as ctx:
        with pytest.raises(rtc.RtcError) as ei:
            rtc.rtc_set_mvm_tuning(ctx, kernel=rtc.RTC_MVM_STREAMED)
        assert ei.value.status == rtc.RTC_E_UNSUPPORTED
