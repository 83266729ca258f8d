"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects invalid configurations before touching a device."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_1805_07254_amd import rtc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def _declared():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(rtc_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = rtc.load_library()
    names = _declared()
    assert "rtc_frame_batch" in names and len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(rtc._SIGNATURES), "binding and header disagree"


def test_abi_version():
    assert rtc.rtc_abi_version() == rtc.RTC_ABI_VERSION


def _cfg(**kw):
    mask = kw.pop("mask", np.ones((4, 4), np.uint8))
    base = dict(abi_version=rtc.RTC_ABI_VERSION, n_sub_x=mask.shape[1], n_sub_y=mask.shape[0], n_pix=4,
                n_act=5, thr_mode=1, cm_dtype=0, gain=0.4, leak=1.0, cmd_min=-math.inf, cmd_max=math.inf,
                device=0)
    base.update(kw)
    m = np.ascontiguousarray(mask)
    c = rtc.rtc_config(base["abi_version"], base["n_sub_x"], base["n_sub_y"], base["n_pix"],
                       m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), base["n_act"], base["thr_mode"],
                       base["cm_dtype"], base["gain"], base["leak"], base["cmd_min"], base["cmd_max"],
                       base["device"])
    return c, m


@pytest.mark.parametrize("kw,status,text", [
    (dict(abi_version=99), rtc.RTC_E_ARG, "abi_version"),
    (dict(n_sub_x=0), rtc.RTC_E_ARG, "n_sub"),
    (dict(n_pix=33), rtc.RTC_E_ARG, "n_pix"),
    (dict(n_act=0), rtc.RTC_E_ARG, "n_act"),
    (dict(thr_mode=3), rtc.RTC_E_ARG, "thr_mode"),
    (dict(thr_mode=-1), rtc.RTC_E_ARG, "thr_mode"),
    (dict(cm_dtype=7), rtc.RTC_E_ARG, "cm_dtype"),
    (dict(gain=math.nan), rtc.RTC_E_NONFINITE, "gain"),
    (dict(leak=math.inf), rtc.RTC_E_NONFINITE, "gain"),
    (dict(cmd_min=1.0, cmd_max=-1.0), rtc.RTC_E_ARG, "cmd_min"),
    (dict(mask=np.zeros((3, 3), np.uint8)), rtc.RTC_E_ARG, "no active"),
    (dict(device=-1), rtc.RTC_E_ARG, "device"),
])
def test_init_rejects_invalid_config_without_a_device(kw, status, text):
    lib = rtc.load_library()
    cfg, _keep = _cfg(**kw)
    out = ctypes.c_void_p(12345)
    st = lib.rtc_init(ctypes.byref(cfg), ctypes.byref(out))
    assert st == status
    assert text in lib.rtc_error_string(None).decode()
    assert out.value == 12345, "output must be untouched on error"


def test_null_arguments():
    lib = rtc.load_library()
    assert lib.rtc_init(None, None) == rtc.RTC_E_ARG
    for name in ["rtc_reset", "rtc_get_state", "rtc_set_state", "rtc_frame", "rtc_load_calib"]:
        fn = getattr(lib, name)
        args = [None] * len(fn.argtypes)
        if name == "rtc_load_calib":
            args[3] = 1.0
        assert fn(*args) == rtc.RTC_E_ARG
    assert lib.rtc_n_valid(None) == -1 and lib.rtc_n_act(None) == -1
    lib.rtc_destroy(None)


def test_row_split_entry_points_reject_null_context():
    lib = rtc.load_library()
    assert lib.rtc_set_row_split(None, 0, None) == rtc.RTC_E_ARG
    assert lib.rtc_get_row_split(None, None, None, 0) == rtc.RTC_E_ARG
    assert lib.rtc_balance_rows(None, 8, None, 0, None, None, None, None) == rtc.RTC_E_ARG


def test_valid_config_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = rtc.load_library()
    cfg, _keep = _cfg()
    out = ctypes.c_void_p()
    assert lib.rtc_init(ctypes.byref(cfg), ctypes.byref(out)) == rtc.RTC_E_DEVICE
    assert out.value is None
    with pytest.raises(rtc.RtcError) as ei:
        rtc.rtc_init(np.ones((2, 2), np.uint8), 4, 3)
    assert ei.value.status == rtc.RTC_E_DEVICE


def _multi(sensors, **kw):
    base = dict(abi_version=rtc.RTC_ABI_VERSION, n_act=5, thr_mode=1, cm_dtype=0, gain=0.4, leak=1.0,
                cmd_min=-math.inf, cmd_max=math.inf, device=0)
    base.update(kw)
    keep = [np.ascontiguousarray(m, np.uint8) for m, _ in sensors]
    arr = (rtc.rtc_wfs * max(len(keep), 1))()
    for w, (m, (_, n)) in enumerate(zip(keep, sensors)):
        arr[w] = rtc.rtc_wfs(m.shape[1], m.shape[0], n, m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    cfg = rtc.rtc_multi_config(base["abi_version"], kw.get("n_wfs", len(keep)), arr, base["n_act"],
                               base["thr_mode"], base["cm_dtype"], base["gain"], base["leak"], base["cmd_min"],
                               base["cmd_max"], base["device"])
    return cfg, (keep, arr)


@pytest.mark.parametrize("sensors,kw,status,text", [
    ([(np.ones((4, 4)), 4)], dict(n_wfs=0), rtc.RTC_E_ARG, "n_wfs"),
    ([(np.ones((4, 4)), 4)], dict(n_wfs=65), rtc.RTC_E_ARG, "n_wfs"),
    ([(np.ones((4, 4)), 4), (np.zeros((3, 3)), 6)], {}, rtc.RTC_E_ARG, "no active"),
    ([(np.ones((4, 4)), 4), (np.ones((2, 2)), 33)], {}, rtc.RTC_E_ARG, "n_pix"),
    ([(np.ones((4096, 4096)), 16), (np.ones((4, 4)), 4)], {}, rtc.RTC_E_ARG, "2^31"),
    ([(np.ones((4, 4)), 4), (np.ones((2, 2)), 6)], dict(abi_version=7), rtc.RTC_E_ARG, "abi_version"),
    ([(np.ones((4, 4)), 4), (np.ones((2, 2)), 6)], dict(thr_mode=9), rtc.RTC_E_ARG, "thr_mode"),
])
def test_init_multi_rejects_invalid_config_without_a_device(sensors, kw, status, text):
    lib = rtc.load_library()
    cfg, _keep = _multi(sensors, **kw)
    out = ctypes.c_void_p(12345)
    assert lib.rtc_init_multi(ctypes.byref(cfg), ctypes.byref(out)) == status
    assert text in lib.rtc_error_string(None).decode()
    assert out.value == 12345
    assert lib.rtc_init_multi(None, ctypes.byref(out)) == rtc.RTC_E_ARG


def test_valid_multi_config_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(rtc.RtcError) as ei:
        rtc.rtc_init_multi([(np.ones((4, 4)), 4), (np.ones((2, 2)), 6)], 9)
    assert ei.value.status == rtc.RTC_E_DEVICE
    assert rtc.load_library().rtc_frame_elems(None) == -1


def test_mlp_create_rejects_bad_sizes_and_reports_no_device():
    lib = rtc.load_library()
    out = ctypes.c_void_p(777)
    assert lib.rtc_mlp_create(0, 4, 4, 8, 0, ctypes.byref(out)) == rtc.RTC_E_ARG
    assert b"sizes" in lib.rtc_mlp_error_string(None)
    assert lib.rtc_mlp_create(4, 4, 4, 1 << 17, 0, ctypes.byref(out)) == rtc.RTC_E_ARG
    assert out.value == 777
    import torch
    if not torch.cuda.is_available():
        assert lib.rtc_mlp_create(4, 4, 4, 8, 0, ctypes.byref(out)) == rtc.RTC_E_DEVICE
    assert lib.rtc_pred_create(None, 1, 1, 1, 1, None, None, None, None, 0.4, ctypes.byref(out)) == rtc.RTC_E_ARG
    mode = ctypes.c_int32(-1)
    assert lib.rtc_pred_last_batch_mode(None, ctypes.byref(mode)) == rtc.RTC_E_ARG and mode.value == -1
    lib.rtc_mlp_destroy(None)
    lib.rtc_pred_destroy(None)
