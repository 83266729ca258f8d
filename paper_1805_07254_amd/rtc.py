"""Thin ctypes binding of ``librtc.so`` (C ABI in ``include/rtc.h``).

Same entry-point names as the C library; the wrappers only check and marshal
arguments (host arrays -> pointers, device tensors -> ``data_ptr()``, torch
streams -> ``hipStream_t``).  Every step of the frame runs in the library's HIP
kernels; there is no host fallback: if ``librtc.so`` is missing, loading fails.
"""
from __future__ import annotations

import ctypes
import math
import os
import weakref
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtc.so")

RTC_ABI_VERSION = 1
RTC_OK, RTC_E_ARG, RTC_E_STATE, RTC_E_NOMEM, RTC_E_DEVICE, RTC_E_NONFINITE, RTC_E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
RTC_THR_NONE, RTC_THR_SUBTRACT, RTC_THR_ZERO = 0, 1, 2
RTC_CM_F32, RTC_CM_F16, RTC_CM_BF16, RTC_CM_FP8E4M3 = 0, 1, 2, 3
CM_DTYPES = {"f32": RTC_CM_F32, "f16": RTC_CM_F16, "bf16": RTC_CM_BF16, "fp8e4m3": RTC_CM_FP8E4M3}
STATUS_NAMES = {0: "RTC_OK", -1: "RTC_E_ARG", -2: "RTC_E_STATE", -3: "RTC_E_NOMEM",
                -4: "RTC_E_DEVICE", -5: "RTC_E_NONFINITE", -6: "RTC_E_UNSUPPORTED"}


class RtcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class rtc_config(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("n_sub_x", ctypes.c_int32), ("n_sub_y", ctypes.c_int32),
                ("n_pix", ctypes.c_int32), ("subap_mask", ctypes.POINTER(ctypes.c_uint8)),
                ("n_act", ctypes.c_int32), ("thr_mode", ctypes.c_int32), ("cm_dtype", ctypes.c_int32),
                ("gain", ctypes.c_float), ("leak", ctypes.c_float), ("cmd_min", ctypes.c_float),
                ("cmd_max", ctypes.c_float), ("device", ctypes.c_int32)]


class rtc_wfs(ctypes.Structure):
    _fields_ = [("n_sub_x", ctypes.c_int32), ("n_sub_y", ctypes.c_int32), ("n_pix", ctypes.c_int32),
                ("subap_mask", ctypes.POINTER(ctypes.c_uint8))]


class rtc_multi_config(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("n_wfs", ctypes.c_int32), ("wfs", ctypes.POINTER(rtc_wfs)),
                ("n_act", ctypes.c_int32), ("thr_mode", ctypes.c_int32), ("cm_dtype", ctypes.c_int32),
                ("gain", ctypes.c_float), ("leak", ctypes.c_float), ("cmd_min", ctypes.c_float),
                ("cmd_max", ctypes.c_float), ("device", ctypes.c_int32)]


RTC_MVM_ROWBLOCK, RTC_MVM_STREAMED = 0, 1
RTC_FRAMES_PER_LAUNCH, RTC_FRAMES_PERSISTENT, RTC_FRAMES_HORIZONTAL = 0, 1, 2


class rtc_mvm_tuning(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("k_split", ctypes.c_int32), ("rows_per_wave", ctypes.c_int32),
                ("unroll", ctypes.c_int32), ("blocks", ctypes.c_int32), ("waves", ctypes.c_int32)]


class rtc_tune_result(ctypes.Structure):
    _fields_ = [("frame_mode", ctypes.c_int32), ("tuning", rtc_mvm_tuning), ("us_per_frame", ctypes.c_float)]


class rtc_pipe_config(ctypes.Structure):
    _fields_ = [("n_workers", ctypes.c_int32), ("full_frame", ctypes.c_int32), ("alloc_ratio", ctypes.c_double),
                ("frame_period_us", ctypes.c_double), ("readout_us", ctypes.c_double),
                ("rows_per_packet", ctypes.c_int32), ("wait_limit_us", ctypes.c_int32),
                ("tail_rows", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_vp, _i32, _i64, _f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
_SIGNATURES = {
    "rtc_init": (_i32, [ctypes.POINTER(rtc_config), ctypes.POINTER(_vp)]),
    "rtc_init_multi": (_i32, [ctypes.POINTER(rtc_multi_config), ctypes.POINTER(_vp)]),
    "rtc_frame_elems": (_i64, [_vp]),
    "rtc_load_calib": (_i32, [_vp, _vp, _vp, _f32, _vp]),
    "rtc_load_calib_multi": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "rtc_graph_capture": (_i32, [_vp, _i32, _vp, _i64, _vp, _vp, _vp, _vp, _vp]),
    "rtc_graph_launch": (_i32, [_vp, _vp]),
    "rtc_get_frame_mode": (_i32, [_vp, ctypes.POINTER(_i32)]),
    "rtc_mlp_create": (_i32, [_i32, _i32, _i32, _i32, _i32, ctypes.POINTER(_vp)]),
    "rtc_mlp_set_params": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "rtc_mlp_get_params": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "rtc_mlp_forward": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "rtc_mlp_loss_grad": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp]),
    "rtc_mlp_get_grads": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "rtc_mlp_adam": (_i32, [_vp, _f32, _f32, _f32, _f32, _i32, _vp]),
    "rtc_mlp_destroy": (None, [_vp]),
    "rtc_mlp_error_string": (ctypes.c_char_p, [_vp]),
    "rtc_pred_create": (_i32, [_vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _f32, ctypes.POINTER(_vp)]),
    "rtc_pred_reset": (_i32, [_vp]),
    "rtc_pred_step": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "rtc_pred_frame_batch": (_i32, [_vp, _vp, _i32, _vp, _i64, _vp, _vp, _vp, _vp]),
    "rtc_pred_last_batch_mode": (_i32, [_vp, _vp]),
    "rtc_pred_destroy": (None, [_vp]),
    "rtc_pred_error_string": (ctypes.c_char_p, [_vp]),
    "rtc_autotune": (_i32, [_vp, _i32, _vp, _i64, _vp, _vp, _i32, ctypes.POINTER(_i32), _vp]),
    "rtc_set_row_split": (_i32, [_vp, _i32, _vp]),
    "rtc_get_row_split": (_i32, [_vp, ctypes.POINTER(_i32), _vp, _i32]),
    "rtc_balance_rows": (_i32, [_vp, _i32, _vp, _i64, _vp, ctypes.POINTER(ctypes.c_float),
                                ctypes.POINTER(ctypes.c_float), _vp]),
    "rtc_pipe_allocation": (_i32, [_i32, _i32, ctypes.c_double, _vp]),
    "rtc_pipe_setup": (_i32, [_vp, ctypes.POINTER(rtc_pipe_config)]),
    "rtc_pipe_info": (_i32, [_vp] + [ctypes.POINTER(_i32)] * 6),
    "rtc_pipe_run": (_i32, [_vp, _i32, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "rtc_load_cmat": (_i32, [_vp, _vp, _i32, _i32, _i64]),
    "rtc_encode_cmat": (_i32, [_i32, _vp, _i32, _i32, _i64, _vp, _vp]),
    "rtc_frame": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "rtc_frame_batch": (_i32, [_vp, _i32, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "rtc_frame_batch_noalloc": (_i32, [_vp, _i32, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "rtc_paced_batch": (_i32, [_vp, _i32, _vp, _i64, _vp, _vp, _vp, _vp, _vp, ctypes.c_double, _vp, _vp, _vp]),
    "rtc_calibrate_centroid": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "rtc_reconstruct_integrate": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "rtc_set_mvm_tuning": (_i32, [_vp, ctypes.POINTER(rtc_mvm_tuning)]),
    "rtc_get_mvm_tuning": (_i32, [_vp, ctypes.POINTER(rtc_mvm_tuning)]),
    "rtc_set_frame_mode": (_i32, [_vp, _i32, _i32]),
    "rtc_sync_check": (_i32, [_vp]),
    "rtc_set_trace": (_i32, [_vp, _vp, _i32, _i32]),
    "rtc_reset": (_i32, [_vp]),
    "rtc_get_state": (_i32, [_vp, _vp]),
    "rtc_set_state": (_i32, [_vp, _vp]),
    "rtc_n_valid": (_i32, [_vp]),
    "rtc_n_act": (_i32, [_vp]),
    "rtc_wall_clock_khz": (_i32, [_vp, ctypes.POINTER(_i64)]),
    "rtc_probe_copy": (_i32, [_vp, _vp, _vp, _i64, _vp]),
    "rtc_probe_read": (_i32, [_vp, _vp, _i64, _vp, _vp]),
    "rtc_error_string": (ctypes.c_char_p, [_vp]),
    "rtc_abi_version": (ctypes.c_uint32, []),
    "rtc_destroy": (None, [_vp]),
}

_lib = None
_handles = weakref.WeakSet()     # live contexts, networks and predictors


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads librtc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with paper_1805_07254_amd.build.build()")
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        if lib.rtc_abi_version() != RTC_ABI_VERSION:
            raise RuntimeError("librtc.so ABI version mismatch")
        _lib = lib
    return _lib


def unload_library() -> None:
    """Closes librtc.so after every context, network and predictor has been
    closed, so that its HIP modules are unregistered now, with the runtime and
    any profiler attached to it still fully alive, rather than by the exit
    handlers of the process.  A later call of the binding loads it again."""
    global _lib
    if _lib is None:
        return
    import gc
    import _ctypes
    gc.collect()
    live = [h for h in list(_handles) if h.handle is not None and getattr(h.handle, "value", h.handle)]
    if live:
        raise RuntimeError(f"unload_library: {len(live)} handle(s) still open; close them first")
    handle, _lib = _lib._handle, None
    _ctypes.dlclose(handle)


class RtcContext:
    """Owning handle of an ``rtc_ctx*``; freed by :meth:`close` or garbage collection."""

    def __init__(self, handle: int, cfg: dict):
        self.handle = ctypes.c_void_p(handle)
        self.cfg = cfg
        _handles.add(self)
        lib = load_library()
        self.n_valid = lib.rtc_n_valid(self.handle)
        self.n_act = lib.rtc_n_act(self.handle)
        self.n_slopes = 2 * self.n_valid
        self.frame_elems = int(lib.rtc_frame_elems(self.handle))   # elements of one frame (set)
        self.n_wfs = len(cfg.get("wfs", [None]))

    def close(self):
        if self.handle is not None and self.handle.value:
            load_library().rtc_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _check(status: int, ctx: Optional[RtcContext]):
    if status != RTC_OK:
        msg = load_library().rtc_error_string(ctx.handle if ctx is not None else None)
        raise RtcError(status, msg.decode() if msg else "")


def _host_ptr(a: Optional[np.ndarray], dtype) -> tuple[Optional[np.ndarray], Optional[int]]:
    if a is None:
        return None, None
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr, arr.ctypes.data


def _dev_ptr(t, dtype_name, numel: int, what: str, ctx: RtcContext, required=True):
    """Device pointer of a torch tensor after checking dtype, device, contiguity and size.

    ``dtype_name`` is a torch dtype name or a tuple of accepted names (same-width
    integer types are interchangeable at the C boundary).  A plain int is taken
    as a raw device address.
    """
    if t is None:
        if required:
            raise ValueError(f"{what} is required")
        return None
    if isinstance(t, int):
        return t
    import torch
    names = (dtype_name,) if isinstance(dtype_name, str) else tuple(dtype_name)
    if t.dtype not in tuple(getattr(torch, n) for n in names):
        raise TypeError(f"{what} must be {' or '.join(names)}, got {t.dtype}")
    if t.device.type != "cuda" or t.device.index != ctx.cfg["device"]:
        raise ValueError(f"{what} must live on cuda:{ctx.cfg['device']}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{what} has {t.numel()} elements, needs {numel}")
    return t.data_ptr()


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# --------------------------------------------------------------------------- API
def rtc_init(subap_mask: np.ndarray, n_pix: int, n_act: int, thr_mode: int = RTC_THR_SUBTRACT,
             cm_dtype=RTC_CM_F32, gain: float = 0.4, leak: float = 1.0,
             cmd_min: float = -math.inf, cmd_max: float = math.inf, device: int = 0,
             abi_version: int = RTC_ABI_VERSION) -> RtcContext:
    lib = load_library()
    if isinstance(cm_dtype, str):
        cm_dtype = CM_DTYPES[cm_dtype]
    mask = np.ascontiguousarray(subap_mask, dtype=np.uint8)
    if mask.ndim != 2:
        raise ValueError("subap_mask must be 2-D [n_sub_y, n_sub_x]")
    cfg = rtc_config(abi_version, mask.shape[1], mask.shape[0], n_pix,
                     mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), n_act, thr_mode, cm_dtype,
                     gain, leak, cmd_min, cmd_max, device)
    out = ctypes.c_void_p()
    st = lib.rtc_init(ctypes.byref(cfg), ctypes.byref(out))
    _check(st, None)
    return RtcContext(out.value, {"n_sub_x": mask.shape[1], "n_sub_y": mask.shape[0], "n_pix": n_pix,
                                  "n_act": n_act, "device": device, "thr_mode": thr_mode, "cm_dtype": cm_dtype,
                                  "gain": gain, "leak": leak})


def rtc_init_multi(sensors, n_act: int, thr_mode: int = RTC_THR_SUBTRACT, cm_dtype=RTC_CM_F32,
                   gain: float = 0.4, leak: float = 1.0, cmd_min: float = -math.inf, cmd_max: float = math.inf,
                   device: int = 0, abi_version: int = RTC_ABI_VERSION) -> RtcContext:
    """sensors: sequence of (subap_mask [n_sub_y, n_sub_x], n_pix) in frame-set order."""
    lib = load_library()
    if isinstance(cm_dtype, str):
        cm_dtype = CM_DTYPES[cm_dtype]
    masks = [np.ascontiguousarray(m, dtype=np.uint8) for m, _ in sensors]
    if any(m.ndim != 2 for m in masks):
        raise ValueError("every subap_mask must be 2-D [n_sub_y, n_sub_x]")
    arr = (rtc_wfs * max(len(masks), 1))()
    for w, (m, (_, n_pix)) in enumerate(zip(masks, sensors)):
        arr[w] = rtc_wfs(m.shape[1], m.shape[0], int(n_pix), m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    cfg = rtc_multi_config(abi_version, len(masks), arr, n_act, thr_mode, cm_dtype, gain, leak, cmd_min, cmd_max,
                           device)
    out = ctypes.c_void_p()
    _check(lib.rtc_init_multi(ctypes.byref(cfg), ctypes.byref(out)), None)
    return RtcContext(out.value, {"wfs": [(m.shape[1], m.shape[0], int(n)) for m, (_, n) in zip(masks, sensors)],
                                  "n_act": n_act, "device": device, "thr_mode": thr_mode, "cm_dtype": cm_dtype,
                                  "gain": gain, "leak": leak})


def rtc_load_calib_multi(ctx: RtcContext, dark: np.ndarray, flat: np.ndarray, thresholds,
                         ref_slopes: Optional[np.ndarray] = None) -> None:
    """dark / flat: the sensors' maps concatenated as a frame set; thresholds: one per sensor."""
    d, dp = _host_ptr(dark, np.float32)
    f, fp = _host_ptr(flat, np.float32)
    if d.size != ctx.frame_elems or f.size != ctx.frame_elems:
        raise ValueError(f"dark/flat must have {ctx.frame_elems} elements")
    t, tp = _host_ptr(np.asarray(thresholds, dtype=np.float32).ravel(), np.float32)
    if t.size != ctx.n_wfs:
        raise ValueError(f"need {ctx.n_wfs} thresholds")
    r, rp = _host_ptr(ref_slopes, np.float32)
    if r is not None and r.size != ctx.n_slopes:
        raise ValueError(f"ref_slopes must have {ctx.n_slopes} elements")
    _check(load_library().rtc_load_calib_multi(ctx.handle, dp, fp, tp, rp), ctx)


def rtc_load_calib(ctx: RtcContext, dark: np.ndarray, flat: np.ndarray, threshold: float,
                   ref_slopes: Optional[np.ndarray] = None) -> None:
    d, dp = _host_ptr(dark, np.float32)
    f, fp = _host_ptr(flat, np.float32)
    if d.size != ctx.frame_elems or f.size != ctx.frame_elems:
        raise ValueError(f"dark/flat must have {ctx.frame_elems} elements")
    r, rp = _host_ptr(ref_slopes, np.float32)
    if r is not None and r.size != ctx.n_slopes:
        raise ValueError(f"ref_slopes must have {ctx.n_slopes} elements")
    _check(load_library().rtc_load_calib(ctx.handle, dp, fp, threshold, rp), ctx)


def rtc_load_cmat(ctx: RtcContext, R: np.ndarray, n_slopes: Optional[int] = None) -> None:
    """R: host [n_act, ld] float32 rows; the first ``n_slopes`` (default ld) columns are used."""
    m, mp = _host_ptr(R, np.float32)
    if m.ndim != 2:
        raise ValueError("R must be 2-D [n_act, ld]")
    ns = m.shape[1] if n_slopes is None else int(n_slopes)
    _check(load_library().rtc_load_cmat(ctx.handle, mp, m.shape[0], ns, m.shape[1]), ctx)


def rtc_encode_cmat(cm_dtype: int, R: np.ndarray):
    """(codes, scales) of a float32 matrix in a reduced storage format (host only)."""
    m, mp = _host_ptr(R, np.float32)
    if m.ndim != 2:
        raise ValueError("R must be 2-D")
    codes = np.empty(m.shape, dtype=np.uint8 if cm_dtype == RTC_CM_FP8E4M3 else np.uint16)
    scales = np.empty(m.shape[0], dtype=np.float32)
    _check(load_library().rtc_encode_cmat(cm_dtype, mp, m.shape[0], m.shape[1], m.shape[1],
                                          codes.ctypes.data, scales.ctypes.data), None)
    return codes, scales


def rtc_frame(ctx: RtcContext, pixels, cmd, slopes=None, recon=None, counts=None, stream=None) -> None:
    lib = load_library()
    _check(lib.rtc_frame(ctx.handle,
                         _dev_ptr(pixels, "uint16", ctx.frame_elems, "pixels", ctx),
                         _dev_ptr(cmd, "float32", ctx.n_act, "cmd", ctx),
                         _dev_ptr(slopes, "float32", ctx.n_slopes, "slopes", ctx, False),
                         _dev_ptr(recon, "float32", ctx.n_act, "recon", ctx, False),
                         _dev_ptr(counts, "int32", ctx.n_valid, "counts", ctx, False),
                         _stream_ptr(stream)), ctx)


def rtc_frame_batch(ctx: RtcContext, n_frames: int, pixels, cmd, slopes=None, recon=None, counts=None,
                    ts=None, frame_stride: Optional[int] = None, stream=None) -> None:
    stride = ctx.frame_elems if frame_stride is None else frame_stride
    need = 0 if n_frames == 0 else (n_frames - 1) * stride + ctx.frame_elems
    _check(load_library().rtc_frame_batch(
        ctx.handle, n_frames,
        _dev_ptr(pixels, "uint16", need, "pixels", ctx),
        stride,
        _dev_ptr(cmd, "float32", n_frames * ctx.n_act, "cmd", ctx),
        _dev_ptr(slopes, "float32", n_frames * ctx.n_slopes, "slopes", ctx, False),
        _dev_ptr(recon, "float32", n_frames * ctx.n_act, "recon", ctx, False),
        _dev_ptr(counts, "int32", n_frames * ctx.n_valid, "counts", ctx, False),
        _dev_ptr(ts, ("uint64", "int64"), 2 * n_frames, "ts", ctx, False),
        _stream_ptr(stream)), ctx)


def rtc_frame_batch_noalloc(ctx: RtcContext, n_frames: int, pixels, cmd, slopes=None, recon=None, counts=None,
                            ts=None, frame_stride: Optional[int] = None, stream=None) -> None:
    """rtc_frame_batch whose kernels use the library's static scratch array."""
    stride = ctx.frame_elems if frame_stride is None else frame_stride
    need = 0 if n_frames == 0 else (n_frames - 1) * stride + ctx.frame_elems
    _check(load_library().rtc_frame_batch_noalloc(
        ctx.handle, n_frames,
        _dev_ptr(pixels, "uint16", need, "pixels", ctx),
        stride,
        _dev_ptr(cmd, "float32", n_frames * ctx.n_act, "cmd", ctx),
        _dev_ptr(slopes, "float32", n_frames * ctx.n_slopes, "slopes", ctx, False),
        _dev_ptr(recon, "float32", n_frames * ctx.n_act, "recon", ctx, False),
        _dev_ptr(counts, "int32", n_frames * ctx.n_valid, "counts", ctx, False),
        _dev_ptr(ts, ("uint64", "int64"), 2 * n_frames, "ts", ctx, False),
        _stream_ptr(stream)), ctx)


def rtc_paced_batch(ctx: RtcContext, n_frames: int, pixels, cmd, period_us: float, slopes=None, recon=None,
                    counts=None, ts=None, frame_stride: Optional[int] = None, stream=None):
    """Host-paced persistent batch; returns (release_ns, done_ns), host int64 [n_frames]."""
    stride = ctx.frame_elems if frame_stride is None else frame_stride
    need = 0 if n_frames == 0 else (n_frames - 1) * stride + ctx.frame_elems
    rel = np.zeros(max(n_frames, 1), np.int64)
    done = np.zeros(max(n_frames, 1), np.int64)
    _check(load_library().rtc_paced_batch(
        ctx.handle, n_frames,
        _dev_ptr(pixels, "uint16", need, "pixels", ctx),
        stride,
        _dev_ptr(cmd, "float32", n_frames * ctx.n_act, "cmd", ctx),
        _dev_ptr(slopes, "float32", n_frames * ctx.n_slopes, "slopes", ctx, False),
        _dev_ptr(recon, "float32", n_frames * ctx.n_act, "recon", ctx, False),
        _dev_ptr(counts, "int32", n_frames * ctx.n_valid, "counts", ctx, False),
        _dev_ptr(ts, ("uint64", "int64"), 2 * n_frames, "ts", ctx, False),
        float(period_us), rel.ctypes.data, done.ctypes.data, _stream_ptr(stream)), ctx)
    return rel[:n_frames], done[:n_frames]


def rtc_calibrate_centroid(ctx: RtcContext, pixels, slopes, counts=None, stream=None) -> None:
    _check(load_library().rtc_calibrate_centroid(
        ctx.handle, _dev_ptr(pixels, "uint16", ctx.frame_elems, "pixels", ctx),
        _dev_ptr(slopes, "float32", ctx.n_slopes, "slopes", ctx),
        _dev_ptr(counts, "int32", ctx.n_valid, "counts", ctx, False), _stream_ptr(stream)), ctx)


def rtc_reconstruct_integrate(ctx: RtcContext, slopes, cmd, recon=None, stream=None) -> None:
    _check(load_library().rtc_reconstruct_integrate(
        ctx.handle, _dev_ptr(slopes, "float32", ctx.n_slopes, "slopes", ctx),
        _dev_ptr(cmd, "float32", ctx.n_act, "cmd", ctx),
        _dev_ptr(recon, "float32", ctx.n_act, "recon", ctx, False), _stream_ptr(stream)), ctx)


TUNING_DEFAULT = {"kernel": RTC_MVM_ROWBLOCK, "k_split": 1, "rows_per_wave": 2, "unroll": 4, "blocks": 0,
                  "waves": 8}
STREAMED_DEFAULT = {**TUNING_DEFAULT, "kernel": RTC_MVM_STREAMED, "rows_per_wave": 2}


def rtc_set_mvm_tuning(ctx: RtcContext, **kw) -> None:
    """Sets the reconstruction launch shape; unspecified fields take that kernel's defaults."""
    unknown = set(kw) - set(TUNING_DEFAULT)
    if unknown:
        raise TypeError(f"unknown tuning fields {sorted(unknown)}")
    base = STREAMED_DEFAULT if kw.get("kernel", RTC_MVM_ROWBLOCK) == RTC_MVM_STREAMED else TUNING_DEFAULT
    t = rtc_mvm_tuning(**{**base, **kw})
    _check(load_library().rtc_set_mvm_tuning(ctx.handle, ctypes.byref(t)), ctx)


def rtc_get_mvm_tuning(ctx: RtcContext) -> dict:
    t = rtc_mvm_tuning()
    _check(load_library().rtc_get_mvm_tuning(ctx.handle, ctypes.byref(t)), ctx)
    return {name: getattr(t, name) for name, _ in rtc_mvm_tuning._fields_}


def rtc_set_frame_mode(ctx: RtcContext, mode: int, spin_limit: int = 0) -> None:
    _check(load_library().rtc_set_frame_mode(ctx.handle, mode, spin_limit), ctx)


def rtc_set_trace(ctx: RtcContext, trace=None, max_frames: int = 0, n_groups: int = 1) -> None:
    """Stage stamps of persistent batches into a device tensor [max_frames, n_groups, 8] (int64/uint64)."""
    ptr = (_dev_ptr(trace, ("uint64", "int64"), 8 * max_frames * n_groups, "trace", ctx, False)
           if max_frames else None)
    _check(load_library().rtc_set_trace(ctx.handle, ptr, max_frames, n_groups), ctx)


def rtc_sync_check(ctx: RtcContext) -> None:
    _check(load_library().rtc_sync_check(ctx.handle), ctx)


def rtc_reset(ctx: RtcContext) -> None:
    _check(load_library().rtc_reset(ctx.handle), ctx)


def rtc_get_state(ctx: RtcContext) -> np.ndarray:
    out = np.empty(ctx.n_act, dtype=np.float32)
    _check(load_library().rtc_get_state(ctx.handle, out.ctypes.data), ctx)
    return out


def rtc_set_state(ctx: RtcContext, cmd: np.ndarray) -> None:
    c, cp = _host_ptr(cmd, np.float32)
    if c.size != ctx.n_act:
        raise ValueError(f"state must have {ctx.n_act} elements")
    _check(load_library().rtc_set_state(ctx.handle, cp), ctx)


def rtc_wall_clock_khz(ctx: RtcContext) -> int:
    out = ctypes.c_int64()
    _check(load_library().rtc_wall_clock_khz(ctx.handle, ctypes.byref(out)), ctx)
    return out.value


def _dev_bytes(t, n_bytes: int, what: str, ctx: RtcContext) -> int:
    """Device pointer of a contiguous torch tensor of any dtype holding at least n_bytes."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    if t.device.type != "cuda" or t.device.index != ctx.cfg["device"]:
        raise ValueError(f"{what} must live on cuda:{ctx.cfg['device']}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if t.numel() * t.element_size() < n_bytes:
        raise ValueError(f"{what} holds {t.numel() * t.element_size()} bytes, needs {n_bytes}")
    return t.data_ptr()


def _probe_size(n_bytes: int) -> int:
    n_bytes = int(n_bytes)
    if n_bytes < 0 or n_bytes % 16:
        raise ValueError("n_bytes must be a non-negative multiple of 16")
    return n_bytes


def rtc_probe_copy(ctx: RtcContext, src, dst, n_bytes: int, stream=None) -> None:
    n_bytes = _probe_size(n_bytes)
    _check(load_library().rtc_probe_copy(ctx.handle, _dev_bytes(src, n_bytes, "src", ctx),
                                         _dev_bytes(dst, n_bytes, "dst", ctx), n_bytes, _stream_ptr(stream)), ctx)


def rtc_probe_read(ctx: RtcContext, src, n_bytes: int, out, stream=None) -> None:
    n_bytes = _probe_size(n_bytes)
    _check(load_library().rtc_probe_read(ctx.handle, _dev_bytes(src, n_bytes, "src", ctx), n_bytes,
                                         _dev_ptr(out, "float32", 1, "out", ctx), _stream_ptr(stream)), ctx)


def rtc_n_valid(ctx: RtcContext) -> int:
    return load_library().rtc_n_valid(ctx.handle)


def rtc_n_act(ctx: RtcContext) -> int:
    return load_library().rtc_n_act(ctx.handle)


def rtc_error_string(ctx: Optional[RtcContext]) -> str:
    s = load_library().rtc_error_string(ctx.handle if ctx is not None else None)
    return s.decode() if s else ""


def rtc_abi_version() -> int:
    return load_library().rtc_abi_version()


def rtc_destroy(ctx: RtcContext) -> None:
    ctx.close()


def rtc_graph_capture(ctx: RtcContext, n_frames: int, pixels, cmd, slopes=None, recon=None, counts=None, ts=None,
                      frame_stride: Optional[int] = None) -> None:
    """Records rtc_frame_batch with these buffers into the context's graph."""
    stride = ctx.frame_elems if frame_stride is None else frame_stride
    need = 0 if n_frames == 0 else (n_frames - 1) * stride + ctx.frame_elems
    _check(load_library().rtc_graph_capture(
        ctx.handle, n_frames, _dev_ptr(pixels, "uint16", need, "pixels", ctx), stride,
        _dev_ptr(cmd, "float32", n_frames * ctx.n_act, "cmd", ctx),
        _dev_ptr(slopes, "float32", n_frames * ctx.n_slopes, "slopes", ctx, False),
        _dev_ptr(recon, "float32", n_frames * ctx.n_act, "recon", ctx, False),
        _dev_ptr(counts, "int32", n_frames * ctx.n_valid, "counts", ctx, False),
        _dev_ptr(ts, ("uint64", "int64"), 2 * n_frames, "ts", ctx, False)), ctx)


def rtc_graph_launch(ctx: RtcContext, stream=None) -> None:
    _check(load_library().rtc_graph_launch(ctx.handle, _stream_ptr(stream)), ctx)


def rtc_autotune(ctx: RtcContext, n_frames: int, pixels, cmd, frame_stride: Optional[int] = None,
                 stream=None) -> list:
    """Times the candidate frame modes / launch shapes, keeps the fastest; returns every candidate's result."""
    stride = ctx.frame_elems if frame_stride is None else frame_stride
    need = (n_frames - 1) * stride + ctx.frame_elems
    res = (rtc_tune_result * 64)()
    n = ctypes.c_int32(0)
    _check(load_library().rtc_autotune(ctx.handle, n_frames, _dev_ptr(pixels, "uint16", need, "pixels", ctx), stride,
                                       _dev_ptr(cmd, "float32", n_frames * ctx.n_act, "cmd", ctx), res, 64,
                                       ctypes.byref(n), _stream_ptr(stream)), ctx)
    out = []
    for r in res[:min(n.value, 64)]:
        out.append({"frame_mode": r.frame_mode, "us_per_frame": r.us_per_frame,
                    "tuning": {name: getattr(r.tuning, name) for name, _ in rtc_mvm_tuning._fields_}})
    return out


def rtc_set_row_split(ctx: RtcContext, row_start=None) -> None:
    """Rows [row_start[b], row_start[b+1]) for workgroup b of persistent launches of len(row_start) - 1
    workgroups; None restores the equal split."""
    if row_start is None:
        _check(load_library().rtc_set_row_split(ctx.handle, 0, None), ctx)
        return
    rs = np.ascontiguousarray(row_start, dtype=np.int32)
    _check(load_library().rtc_set_row_split(ctx.handle, int(rs.size) - 1, rs.ctypes.data), ctx)


def rtc_get_row_split(ctx: RtcContext) -> Optional[np.ndarray]:
    """The current row split (None: equal split)."""
    g = ctypes.c_int32(0)
    _check(load_library().rtc_get_row_split(ctx.handle, ctypes.byref(g), None, 0), ctx)
    if g.value == 0:
        return None
    out = np.zeros(g.value + 1, dtype=np.int32)
    _check(load_library().rtc_get_row_split(ctx.handle, ctypes.byref(g), out.ctypes.data, out.size), ctx)
    return out


def rtc_balance_rows(ctx: RtcContext, n_frames: int, pixels, cmd, frame_stride: Optional[int] = None,
                     stream=None) -> dict:
    """Measured row split of persistent batches; returns the mean frame times with the equal and the measured
    split (the faster is kept)."""
    stride = ctx.frame_elems if frame_stride is None else frame_stride
    need = (n_frames - 1) * stride + ctx.frame_elems
    eq, sp = ctypes.c_float(-1.0), ctypes.c_float(-1.0)
    _check(load_library().rtc_balance_rows(ctx.handle, n_frames, _dev_ptr(pixels, "uint16", need, "pixels", ctx),
                                           stride, _dev_ptr(cmd, "float32", n_frames * ctx.n_act, "cmd", ctx),
                                           ctypes.byref(eq), ctypes.byref(sp), _stream_ptr(stream)), ctx)
    return {"us_equal": eq.value, "us_split": sp.value, "kept": "split" if rtc_get_row_split(ctx) is not None
            else "equal"}


def rtc_pipe_allocation(n_subaps: int, n_workers: int, ratio: float) -> np.ndarray:
    """Linearly decreasing subaperture counts per worker (host only)."""
    counts = np.zeros(max(n_workers, 1), dtype=np.int32)
    _check(load_library().rtc_pipe_allocation(n_subaps, n_workers, float(ratio), counts.ctypes.data), None)
    return counts


def rtc_pipe_setup(ctx: RtcContext, n_workers: int = 0, full_frame: bool = False, alloc_ratio: float = 1.0,
                   frame_period_us: float = 1000.0, readout_us: Optional[float] = None,
                   rows_per_packet: int = 2, wait_limit_us: int = 0, tail_rows: int = 0) -> None:
    cfg = rtc_pipe_config(n_workers=n_workers, full_frame=1 if full_frame else 0, alloc_ratio=float(alloc_ratio),
                          frame_period_us=float(frame_period_us),
                          readout_us=float(frame_period_us if readout_us is None else readout_us),
                          rows_per_packet=rows_per_packet, wait_limit_us=wait_limit_us, tail_rows=tail_rows,
                          reserved=0)
    _check(load_library().rtc_pipe_setup(ctx.handle, ctypes.byref(cfg)), ctx)


def rtc_pipe_info(ctx: RtcContext) -> dict:
    v = [ctypes.c_int32(0) for _ in range(6)]
    _check(load_library().rtc_pipe_info(ctx.handle, *[ctypes.byref(x) for x in v]), ctx)
    return {"n_workers": v[0].value, "lds_cols": v[1].value, "image_rows": v[2].value, "max_subaps": v[3].value,
            "n_tail": v[4].value, "n_owners": v[5].value}


def rtc_pipe_run(ctx: RtcContext, n_frames: int, frames, cmd, slopes=None, recon=None, counts=None, cam_ts=None,
                 worker_ts=None, frame_stride: Optional[int] = None, stream=None) -> None:
    stride = ctx.frame_elems if frame_stride is None else frame_stride
    need = 0 if n_frames == 0 else (n_frames - 1) * stride + ctx.frame_elems
    n_workers = rtc_pipe_info(ctx)["n_workers"] if worker_ts is not None else 0
    _check(load_library().rtc_pipe_run(
        ctx.handle, n_frames,
        _dev_ptr(frames, "uint16", need, "frames", ctx),
        stride,
        _dev_ptr(cmd, "float32", n_frames * ctx.n_act, "cmd", ctx),
        _dev_ptr(slopes, "float32", n_frames * ctx.n_slopes, "slopes", ctx, False),
        _dev_ptr(recon, "float32", n_frames * ctx.n_act, "recon", ctx, False),
        _dev_ptr(counts, "int32", n_frames * ctx.n_valid, "counts", ctx, False),
        _dev_ptr(cam_ts, ("uint64", "int64"), 4 * n_frames, "cam_ts", ctx, False),
        _dev_ptr(worker_ts, ("uint64", "int64"), 2 * n_frames * n_workers, "worker_ts", ctx, False),
        _stream_ptr(stream)), ctx)


def rtc_get_frame_mode(ctx: RtcContext) -> int:
    m = ctypes.c_int32(-1)
    _check(load_library().rtc_get_frame_mode(ctx.handle, ctypes.byref(m)), ctx)
    return m.value


# ---------------------------------------------------------------------------
# learned predictor (include/rtc_mlp.h)
def _mcheck(status: int, handle, err_fn: str):
    if status != RTC_OK:
        msg = getattr(load_library(), err_fn)(handle)
        raise RtcError(status, msg.decode() if msg else "")


class MlpNet:
    """Owning handle of an ``rtc_mlp*`` (n_in -> n_hidden GELU -> n_out)."""

    def __init__(self, n_in: int, n_hidden: int, n_out: int, max_batch: int, device: int = 0):
        out = _vp()
        _mcheck(load_library().rtc_mlp_create(n_in, n_hidden, n_out, max_batch, device, ctypes.byref(out)), None,
                "rtc_mlp_error_string")
        self.handle = out
        _handles.add(self)
        self.n_in, self.n_hidden, self.n_out, self.max_batch, self.device = n_in, n_hidden, n_out, max_batch, device

    def _chk(self, st):
        _mcheck(st, self.handle, "rtc_mlp_error_string")

    def _shapes(self):
        return [(self.n_hidden, self.n_in), (self.n_hidden,), (self.n_out, self.n_hidden), (self.n_out,)]

    def set_params(self, W1, b1, W2, b2) -> None:
        arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (W1, b1, W2, b2)]
        for a, shp in zip(arrs, self._shapes()):
            if a.shape != shp:
                raise ValueError(f"parameter shape {a.shape} != {shp}")
        self._chk(load_library().rtc_mlp_set_params(self.handle, *[a.ctypes.data for a in arrs]))

    def get_params(self):
        arrs = [np.empty(shp, np.float32) for shp in self._shapes()]
        self._chk(load_library().rtc_mlp_get_params(self.handle, *[a.ctypes.data for a in arrs]))
        return arrs

    def get_grads(self):
        arrs = [np.empty(shp, np.float32) for shp in self._shapes()]
        self._chk(load_library().rtc_mlp_get_grads(self.handle, *[a.ctypes.data for a in arrs]))
        return arrs

    def _dev(self, t, numel, what):
        import torch
        if t.dtype != torch.float32 or t.device.type != "cuda" or not t.is_contiguous() or t.numel() < numel:
            raise ValueError(f"{what}: need a contiguous float32 device tensor of >= {numel} elements")
        return t.data_ptr()

    def forward(self, batch: int, x, y, stream=None) -> None:
        self._chk(load_library().rtc_mlp_forward(self.handle, batch, self._dev(x, batch * self.n_in, "x"),
                                                 self._dev(y, batch * self.n_out, "y"), _stream_ptr(stream)))

    def loss_grad(self, batch: int, x, t, loss, stream=None) -> None:
        self._chk(load_library().rtc_mlp_loss_grad(self.handle, batch, self._dev(x, batch * self.n_in, "x"),
                                                   self._dev(t, batch * self.n_out, "t"), self._dev(loss, 1, "loss"),
                                                   _stream_ptr(stream)))

    def adam(self, lr: float, step: int, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
             stream=None) -> None:
        self._chk(load_library().rtc_mlp_adam(self.handle, lr, beta1, beta2, eps, step, _stream_ptr(stream)))

    def close(self):
        if self.handle is not None and self.handle.value:
            load_library().rtc_mlp_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Predictor:
    """Owning handle of an ``rtc_pred*`` (predictive feed-forward); keeps its network alive."""

    def __init__(self, net: MlpNet, history: int, P, PD, mean, std, gain: float):
        P, PD, mean, std = (np.ascontiguousarray(a, dtype=np.float32) for a in (P, PD, mean, std))
        n_modes, n_slopes = P.shape
        n_act = PD.shape[1]
        if PD.shape != (n_modes, n_act) or mean.shape != (n_modes,) or std.shape != (n_modes,):
            raise ValueError("P [n_modes, n_slopes], PD [n_modes, n_act], mean/std [n_modes]")
        out = _vp()
        _mcheck(load_library().rtc_pred_create(net.handle, history, n_modes, n_slopes, n_act, P.ctypes.data,
                                               PD.ctypes.data, mean.ctypes.data, std.ctypes.data, gain,
                                               ctypes.byref(out)), None, "rtc_pred_error_string")
        self.handle, self.net = out, net
        _handles.add(self)
        self.history, self.n_modes, self.n_slopes, self.n_act = history, n_modes, n_slopes, n_act

    def _chk(self, st):
        _mcheck(st, self.handle, "rtc_pred_error_string")

    def reset(self) -> None:
        self._chk(load_library().rtc_pred_reset(self.handle))

    def step(self, slopes, cmd_prev, slopes_out, modes=None, stream=None) -> None:
        """slopes_out = slopes + P^T (forecast change) / gain, to be fed to the integrator."""
        ptr = lambda t, n, w: MlpNet._dev(self.net, t, n, w)
        self._chk(load_library().rtc_pred_step(self.handle, ptr(slopes, self.n_slopes, "slopes"),
                                               ptr(cmd_prev, self.n_act, "cmd_prev"),
                                               ptr(slopes_out, self.n_slopes, "slopes_out"),
                                               None if modes is None else ptr(modes, 2 * self.n_modes, "modes"),
                                               _stream_ptr(stream)))

    def frame_batch(self, ctx: RtcContext, n_frames: int, pixels, cmd, slopes=None, ts=None,
                    frame_stride: Optional[int] = None, stream=None) -> None:
        """n_frames predictive frames of ctx (calibration, this step, reconstruction and integrator)."""
        stride = ctx.frame_elems if frame_stride is None else frame_stride
        need = 0 if n_frames == 0 else (n_frames - 1) * stride + ctx.frame_elems
        self._chk(load_library().rtc_pred_frame_batch(
            ctx.handle, self.handle, n_frames, _dev_ptr(pixels, "uint16", need, "pixels", ctx), stride,
            _dev_ptr(cmd, "float32", n_frames * ctx.n_act, "cmd", ctx),
            _dev_ptr(slopes, "float32", n_frames * ctx.n_slopes, "slopes", ctx, False),
            _dev_ptr(ts, ("uint64", "int64"), 2 * n_frames, "ts", ctx, False), _stream_ptr(stream)))

    def last_batch_mode(self) -> int:
        """RTC_FRAMES_PERSISTENT or RTC_FRAMES_PER_LAUNCH: how the last frame_batch ran."""
        out = ctypes.c_int32()
        self._chk(load_library().rtc_pred_last_batch_mode(self.handle, ctypes.byref(out)))
        return out.value

    def close(self):
        if self.handle is not None and self.handle.value:
            load_library().rtc_pred_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
