"""rtc_frame_batch_noalloc: the frame batch whose kernels use the library's
static scratch array, against rtc_frame_batch on twin contexts."""
import numpy as np
import pytest

from _closedloop import oracle_closed_loop
from _gpu_helpers import _ctx_for, _dev, check_parity
from aosim import ELT, TINY, Scenario, geometry

torch = pytest.importorskip("torch")
from paper_1805_07254_amd import rtc  # noqa: E402

pytestmark = pytest.mark.gpu

MODES = {"per_launch": rtc.RTC_FRAMES_PER_LAUNCH, "persistent": rtc.RTC_FRAMES_PERSISTENT,
         "horizontal": rtc.RTC_FRAMES_HORIZONTAL}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rtc.load_library()


@pytest.fixture(scope="module")
def loops():
    elt, tiny = Scenario(ELT), Scenario(TINY)
    return {"elt": (elt,) + oracle_closed_loop(elt, 6), "tiny": (tiny,) + oracle_closed_loop(tiny, 40)}


def _run(ctx, frames, call):
    F = frames.shape[0]
    pix = _dev(frames.reshape(F, -1))
    out = {"cmd": torch.empty(F * ctx.n_act, dtype=torch.float32, device="cuda:0"),
           "slopes": torch.empty(F * ctx.n_slopes, dtype=torch.float32, device="cuda:0"),
           "recon": torch.empty(F * ctx.n_act, dtype=torch.float32, device="cuda:0"),
           "counts": torch.empty(F * ctx.n_valid, dtype=torch.int32, device="cuda:0"),
           "ts": torch.zeros(2 * F, dtype=torch.int64, device="cuda:0")}
    call(ctx, F, pix, out["cmd"], out["slopes"], out["recon"], out["counts"], out["ts"])
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().reshape(F, -1) for k, v in out.items()}


def _pair(sc, mode, fmt, tuning):
    """A context for the static-scratch call in `mode` and a twin for
    rtc_frame_batch (horizontal contexts run the row split there, so the twin
    runs persistent)."""
    a = _ctx_for(sc, cm_dtype=fmt)
    b = _ctx_for(sc, cm_dtype=fmt)
    rtc.rtc_set_frame_mode(a, MODES[mode])
    rtc.rtc_set_frame_mode(b, rtc.RTC_FRAMES_PERSISTENT if mode == "horizontal" else MODES[mode])
    for ctx in (a, b):
        rtc.rtc_set_mvm_tuning(ctx, **tuning)
    return a, b


@pytest.mark.parametrize("mode,fmt,tuning", [
    ("per_launch", "f32", {}),
    ("per_launch", "f32", {"kernel": rtc.RTC_MVM_STREAMED, "k_split": 4, "rows_per_wave": 2}),
    ("persistent", "f32", {}),
    ("persistent", "bf16", {}),
    ("horizontal", "f32", {}),
])
def test_noalloc_batch_equals_frame_batch_on_two_calls(loops, mode, fmt, tuning):
    # first call on the ELT shape, the second on the tiny shape: the array then
    # holds the larger call's contents, which the second call must not see
    for name in ("elt", "tiny"):
        sc, frames, ref = loops[name]
        print(f"noalloc {mode} {fmt} {tuning} on {name}: {frames.shape[0]} frames", flush=True)
        a, b = _pair(sc, mode, fmt, tuning)
        with a, b:
            got = _run(a, frames, rtc.rtc_frame_batch_noalloc)
            want = _run(b, frames, rtc.rtc_frame_batch)
            rtc.rtc_sync_check(a)
            rtc.rtc_sync_check(b)
            state_a, state_b = rtc.rtc_get_state(a), rtc.rtc_get_state(b)
        for key in ("counts", "slopes", "recon", "cmd"):
            assert np.array_equal(got[key], want[key]), f"{name} {mode} {fmt}: {key} differs"
        assert np.array_equal(state_a, state_b)
        assert np.all(got["ts"][:, 1] > got["ts"][:, 0])
        if fmt == "f32":
            check_parity(got, ref, sc.cfg.gain, sc.cfg.leak, what=f"{name} noalloc {mode}")


def test_noalloc_batches_compose_and_continue_from_state(loops):
    sc, frames, ref = loops["tiny"]
    a, b = _pair(sc, "persistent", "f32", {})
    with a, b:
        whole = _run(b, frames, rtc.rtc_frame_batch)
        first = _run(a, frames[:15], rtc.rtc_frame_batch_noalloc)
        second = _run(a, frames[15:], rtc.rtc_frame_batch_noalloc)
        rtc.rtc_sync_check(a)
    assert np.array_equal(np.concatenate([first["cmd"], second["cmd"]]), whole["cmd"])


def test_noalloc_rejects_contexts_beyond_the_static_scratch():
    # 64 split-K partial vectors of 20000 actuators need 5.1 MB, beyond the 4 MiB array
    mask = geometry.subaperture_mask(4, 0.0).astype(np.uint8)
    nv = int(mask.sum())
    n_act = 20000
    rng = np.random.default_rng(3)
    with rtc.rtc_init(mask, 4, n_act) as ctx:
        rtc.rtc_load_calib(ctx, np.zeros((16, 16), np.float32), np.ones((16, 16), np.float32), 1.0)
        rtc.rtc_load_cmat(ctx, rng.standard_normal((n_act, 2 * nv)).astype(np.float32))
        rtc.rtc_set_mvm_tuning(ctx, kernel=rtc.RTC_MVM_STREAMED, k_split=64, rows_per_wave=2)
        pix = _dev(rng.integers(0, 300, size=(1, 256)).astype(np.uint16))
        cmd = torch.empty(n_act, dtype=torch.float32, device="cuda:0")
        with pytest.raises(rtc.RtcError) as ei:
            rtc.rtc_frame_batch_noalloc(ctx, 1, pix, cmd)
        assert ei.value.status == rtc.RTC_E_UNSUPPORTED
        assert "static scratch" in str(ei.value)
        # the same context runs once the partial vectors fit
        rtc.rtc_set_mvm_tuning(ctx, kernel=rtc.RTC_MVM_STREAMED, k_split=8, rows_per_wave=2)
        rtc.rtc_frame_batch_noalloc(ctx, 1, pix, cmd)
        want = torch.empty_like(cmd)
        rtc.rtc_reset(ctx)
        rtc.rtc_frame_batch(ctx, 1, pix, want)
        torch.cuda.synchronize()
        assert torch.equal(cmd, want)
