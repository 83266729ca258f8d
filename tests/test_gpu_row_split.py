"""Measured row split of persistent batches (rtc_set_row_split, rtc_balance_rows).

Each row's sum does not depend on the workgroup that computes it, so any
split must give results bitwise equal to the per-launch mode."""
import numpy as np
import pytest

from _gpu_helpers import _ctx_for, _dev, _gpu_batch
from aosim import ELT, TINY, Scenario, geometry

torch = pytest.importorskip("torch")
from paper_1805_07254_amd import rtc  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rtc.load_library()


def _grid(n_act):
    return min(torch.cuda.get_device_properties(0).multi_processor_count, n_act)


def _skewed_split(n_act, G, seed):
    # uneven shares, every one in [1, 512]
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.5, 1.5, G)
    cnt = np.maximum(1, np.floor(w / w.sum() * (n_act - G)).astype(np.int64) + 1)
    cnt[np.argmax(cnt)] += n_act - cnt.sum()
    assert cnt.min() >= 1 and cnt.max() <= 512 and cnt.sum() == n_act
    return np.concatenate([[0], np.cumsum(cnt)]).astype(np.int32)


def _frames(sc, n):
    return np.stack([sc.frame(i, sc.turbulence_slopes(i)) for i in range(n)])


@pytest.mark.parametrize("name,fmt", [("tiny", "f32"), ("elt", "f32"), ("elt", "bf16")])
def test_any_row_split_is_bitwise_the_per_launch_result(name, fmt):
    sc = Scenario(TINY if name == "tiny" else ELT)
    frames = _frames(sc, 6)
    out = []
    with _ctx_for(sc, cm_dtype=fmt) as ctx:
        out.append(_gpu_batch(ctx, frames))
    with _ctx_for(sc, cm_dtype=fmt) as ctx:
        rtc.rtc_set_frame_mode(ctx, rtc.RTC_FRAMES_PERSISTENT)
        rs = _skewed_split(sc.n_act, _grid(sc.n_act), 5)
        rtc.rtc_set_row_split(ctx, rs)
        assert np.array_equal(rtc.rtc_get_row_split(ctx), rs)
        out.append(_gpu_batch(ctx, frames))
        rtc.rtc_sync_check(ctx)
    for key in out[0]:
        assert np.array_equal(out[0][key], out[1][key]), key


def test_row_split_with_slope_panels_is_bitwise_the_per_launch_result():
    rng = np.random.default_rng(21)
    mask = geometry.subaperture_mask(110, 0.0)
    nv = int(mask.sum())
    n, H, n_act = 10, 1100, 700
    frames = rng.integers(95, 200, size=(3, H, H)).astype(np.uint16)
    dark = rng.uniform(95.0, 105.0, size=(H, H)).astype(np.float32)
    flat = rng.normal(1.0, 0.02, size=(H, H)).astype(np.float32)
    R = (rng.standard_normal((n_act, 2 * nv)) / 100).astype(np.float32)
    out = []
    for split in (False, True):
        with rtc.rtc_init(mask, n, n_act, cm_dtype="bf16") as ctx:
            rtc.rtc_load_calib(ctx, dark, flat, 20.0)
            rtc.rtc_load_cmat(ctx, R)
            if split:
                rtc.rtc_set_frame_mode(ctx, rtc.RTC_FRAMES_PERSISTENT)
                rtc.rtc_set_row_split(ctx, _skewed_split(n_act, _grid(n_act), 6))
            out.append(_gpu_batch(ctx, frames))
            rtc.rtc_sync_check(ctx)
    assert 2 * nv > 16384
    for key in out[0]:
        assert np.array_equal(out[0][key], out[1][key]), key


def test_split_for_another_grid_is_not_used_and_none_restores_equal():
    sc = Scenario(TINY)
    frames = _frames(sc, 4)
    with _ctx_for(sc) as ctx:
        ref = _gpu_batch(ctx, frames)
    with _ctx_for(sc) as ctx:
        rtc.rtc_set_frame_mode(ctx, rtc.RTC_FRAMES_PERSISTENT)
        G = _grid(sc.n_act)
        rtc.rtc_set_row_split(ctx, _skewed_split(sc.n_act, G - 1, 7))   # a grid this context does not launch
        got = _gpu_batch(ctx, frames)
        rtc.rtc_set_row_split(ctx, None)
        assert rtc.rtc_get_row_split(ctx) is None
        got2 = _gpu_batch(ctx, frames[:1])
    for key in ref:
        assert np.array_equal(ref[key], got[key]), key
    assert np.array_equal(ref["slopes"][:1], got2["slopes"])


@pytest.mark.parametrize("bad", ["start", "end", "empty", "too_many", "grid"])
def test_malformed_splits_are_rejected(bad):
    sc = Scenario(TINY)
    n_act = 1100
    with rtc.rtc_init(sc.mask, sc.cfg.n_pix, n_act) as ctx:
        rs = np.linspace(0, n_act, 9).astype(np.int32)
        if bad == "start":
            rs[0] = 1
        elif bad == "end":
            rs[-1] = n_act - 1
        elif bad == "empty":
            rs[3] = rs[2]
        elif bad == "too_many":
            rs = np.array([0, 550, n_act], np.int32)         # 550 rows for one workgroup
        else:
            rs = np.zeros(1026, np.int32)                    # 1025 workgroups
        with pytest.raises(rtc.RtcError) as e:
            rtc.rtc_set_row_split(ctx, rs)
        assert e.value.status == rtc.RTC_E_ARG
        assert rtc.rtc_get_row_split(ctx) is None


def test_balance_rows_keeps_state_and_results():
    sc = Scenario(ELT)
    frames = _frames(sc, 8)
    F = 64
    ring = torch.from_numpy(np.ascontiguousarray(frames.reshape(8, -1)).view(np.int16)).to("cuda:0")
    pix = ring[torch.arange(F, device="cuda:0") % 8].contiguous().view(torch.uint16)
    cmd = torch.empty(F * sc.n_act, dtype=torch.float32, device="cuda:0")
    with _ctx_for(sc) as ctx:
        ref = _gpu_batch(ctx, frames[:4])
    with _ctx_for(sc) as ctx:
        rtc.rtc_set_frame_mode(ctx, rtc.RTC_FRAMES_PERSISTENT)
        state = np.linspace(-1.0, 1.0, sc.n_act).astype(np.float32)
        rtc.rtc_set_state(ctx, state)
        res = rtc.rtc_balance_rows(ctx, F, pix, cmd)
        assert res["us_equal"] > 0 and res["us_split"] > 0
        assert res["kept"] == ("split" if res["us_split"] < res["us_equal"] else "equal")
        assert np.array_equal(rtc.rtc_get_state(ctx), state)
        split = rtc.rtc_get_row_split(ctx)
        if split is not None:
            assert split[0] == 0 and split[-1] == sc.n_act and np.diff(split).min() >= 1
        rtc.rtc_reset(ctx)
        got = _gpu_batch(ctx, frames[:4])
        rtc.rtc_sync_check(ctx)
    for key in ref:
        assert np.array_equal(ref[key], got[key]), key


def test_balance_rows_needs_the_persistent_mode():
    sc = Scenario(TINY)
    with _ctx_for(sc) as ctx:
        pix = _dev(_frames(sc, 4).reshape(4, -1))
        cmd = torch.empty(4 * sc.n_act, dtype=torch.float32, device="cuda:0")
        with pytest.raises(rtc.RtcError) as e:
            rtc.rtc_balance_rows(ctx, 4, pix, cmd)
        assert e.value.status == rtc.RTC_E_STATE
