"""Benchmark of the AO real-time-control frame on one MI355X.

One step = one ELT-scale SCAO frame through the whole hot path (calibration,
centre of gravity, control-matrix x slopes, integrator), FP32, in the
persistent kernel.  Frames run back to back from a device buffer holding one
raw frame per step (copies of a ring of distinct open-loop frames), so every
frame's pixels are read from HBM.  ``value`` is the p50 of the timed frames'
span: the first workgroup's start of the frame to the last workgroup's
command store, from per-frame device time stamps (the paper's latency without
a camera is the frame computation time).  Around it:

  * long runs: whole launches of --roofline-frames frames, timed with HIP
    events on the launch stream (the roofline's device time), with the
    period and span statistics of every frame (p50, p99, RMS and
    peak-to-peak jitter, with and without the first 100 frames);
  * a stage trace of every workgroup, whose last-arrival-to-release time is
    the measured barrier floor of the frame model;
  * a host-paced run: frames released one by one at a fixed period through a
    word of coherent host memory, latency taken on the host from the release
    to the completion word (rtc_paced_batch);
  * the horizontal split, the per-launch mode, the reduced-precision
    matrices, read/copy bandwidth probes;
  * the FP64 oracle on the host's cores (all cores, and one core in a child
    process) as a CPU baseline.

The roofline reports the frames kernel against the FP32 VALU peak (its work
is FMAs on operands kept on chip), with a frame model built from rocprofv3
counters of the committed profile (VALU issue, LDS and L2 bytes, HBM traffic)
plus the measured barrier floor, and the HBM view kept separately.

    python bench.py [--steps 10000] [--warmup 1000]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("ELT-SCAO frame latency p50/p99 + RMS jitter (µs); GEMV GB/s vs HBM/LLC peak")
HBM_PEAK_GBPS = 8000.0
# MI355X: 256 compute units at 2.4 GHz; FP32 FMA without packed math is 64
# lanes per cycle per unit (16 per SIMD), 78.6 TFLOP/s, i.e. one wave64 VALU
# instruction per cycle per unit; LDS 128 bytes per cycle per unit; L2 16
# channels x 128 bytes per cycle per XCD of 32 units = 64 bytes per cycle per
# unit; a TCP-to-L2 read request moves 128 bytes (a 256 MiB copy counts
# 2,097,152 of them)
N_CU = 256
CLK_GHZ = 2.4
VALU_PEAK_TFLOPS = 78.6
LDS_BYTES_PER_CLK = 128
L2_BYTES_PER_CLK_PER_CU = 64
TCP_REQ_BYTES = 128
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "frames_elt_counters.json")
KERNEL_SRCS = [os.path.join(ROOT, "paper_1805_07254_amd", "csrc", f)
               for f in ("rtc_kernels.hip", "rtc_device.h", "rtc_kernels.h")]
FMT_BYTES = {"f32": 4, "f16": 2, "bf16": 2, "fp8e4m3": 1}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """sha256 prefix of the sources of the persistent frame kernel."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def frame_bytes(sc, fmt: str) -> int:
    """Algorithmic bytes of one frame: matrix (+ row scales), valid pixels,
    dark and flat of the valid pixels, slope vector written and read, command
    vector read and written."""
    n_act, n_s, n_v, n_pix = sc.n_act, 2 * sc.n_valid, sc.n_valid, sc.cfg.n_pix
    matrix = n_act * n_s * FMT_BYTES[fmt] + (0 if fmt == "f32" else 4 * n_act)
    return matrix + n_v * n_pix * n_pix * (2 + 8) + 2 * 4 * n_s + 2 * 4 * n_act


def frame_flops(sc) -> int:
    """Algorithmic floating-point operations of one frame: 2 per matrix
    element (multiply-add), 8 per valid pixel (dark subtraction, flat,
    threshold compare and subtract, three weighted sums), 4 per actuator
    (integrator multiply-add, clamp)."""
    n_pix = sc.cfg.n_pix
    return 2 * sc.n_act * 2 * sc.n_valid + 8 * sc.n_valid * n_pix * n_pix + 4 * sc.n_act


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10000)
    p.add_argument("--warmup", type=int, default=1000)
    p.add_argument("--launch-frames", type=int, default=10000, help="frames per persistent launch")
    p.add_argument("--ring", type=int, default=128, help="distinct raw frames (repeated through the buffer)")
    p.add_argument("--mvm-kernel", type=int, default=0, help="0 = row-block, 1 = streamed")
    p.add_argument("--k-split", type=int, default=1)
    p.add_argument("--rows-per-wave", type=int, default=2)
    p.add_argument("--unroll", type=int, default=4)
    p.add_argument("--blocks", type=int, default=0)
    p.add_argument("--waves", type=int, default=8)
    p.add_argument("--kernel-reps", type=int, default=2000)
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--variants", default="f16,bf16,fp8e4m3",
                   help="reduced-precision matrix formats also timed (comma list, none = no variant)")
    p.add_argument("--variant-steps", type=int, default=2000)
    p.add_argument("--workload", default="elt-scao", choices=["elt-scao", "elt-multi", "elt-predict", "elt-pipe"],
                   help="elt-scao: the single-sensor ELT frame (default); elt-multi: six 74x74 and three 16x16 "
                        "sensors reconstructed by one BF16 matrix")
    p.add_argument("--balance-rows", action="store_true",
                   help="headline: measured row split of the persistent workgroups (rtc_balance_rows) before timing")
    p.add_argument("--multi-steps", type=int, default=5000)
    p.add_argument("--multi-ring", type=int, default=4, help="distinct multi-sensor frame sets")
    p.add_argument("--multi-dtype", default="bf16")
    p.add_argument("--pipe-frames", type=int, default=1000, help="camera frames per pixel-stream mode (elt-pipe)")
    p.add_argument("--pipe-period-us", type=float, default=1000.0, help="camera frame period (elt-pipe)")
    p.add_argument("--pipe-readout-us", type=float, default=1000.0, help="camera readout time (elt-pipe)")
    p.add_argument("--pred-frames", type=int, default=200000, help="closed-loop training frames (elt-predict)")
    p.add_argument("--pred-modes", type=int, default=500)
    p.add_argument("--pred-hidden", type=int, default=1024)
    p.add_argument("--pred-history", type=int, default=5)
    p.add_argument("--pred-epochs", type=int, default=6)
    p.add_argument("--pred-batch", type=int, default=512)
    p.add_argument("--pred-latency-frames", type=int, default=2000,
                   help="ELT pixel frames timed plain and predictive (elt-predict)")
    p.add_argument("--roofline-frames", type=int, default=10000, help="frames per roofline launch")
    p.add_argument("--roofline-launches", type=int, default=2,
                   help="launches of --roofline-frames frames without time stamps (the roofline's device time)")
    p.add_argument("--stats-launches", type=int, default=3,
                   help="launches of --roofline-frames frames with time stamps (latency distribution)")
    p.add_argument("--trace-frames", type=int, default=1000, help="frames of the all-workgroup stage trace")
    p.add_argument("--paced-frames", type=int, default=2000, help="host-paced frames (0 = none)")
    p.add_argument("--paced-period-us", type=float, default=1000.0)
    p.add_argument("--horizontal-steps", type=int, default=2000, help="frames timed in the horizontal split")
    p.add_argument("--probes", default="35MB,70MB,140MB,488MB,2GB", help="read-probe working sets (comma list, none = no probe)")
    p.add_argument("--cpu-leg", type=int, default=None, help=argparse.SUPPRESS)
    return p.parse_args()


def cpu_baseline(sc, ring_host, seconds: float) -> dict:
    """The FP64 oracle timed per frame on this host's cores (a bounded sample)."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        blas_threads = 1
    cfg = sc.cfg
    fo = oracle.FrameOracle(sc.mask, cfg.n_pix, sc.dark, sc.flat, cfg.threshold, sc.control_matrix,
                            cfg.gain, cfg.leak)
    c = np.zeros(sc.n_act)
    times = []
    t_end = time.perf_counter() + seconds
    k = 0
    while time.perf_counter() < t_end or k < 3:
        t0 = time.perf_counter_ns()
        out = fo(ring_host[k % len(ring_host)], c)
        times.append((time.perf_counter_ns() - t0) / 1e3)
        c = out["cmd"]
        k += 1
    t = np.asarray(times[1:] if len(times) > 1 else times)
    cores = min(int(blas_threads), len(os.sched_getaffinity(0)))
    return {"value": float(np.median(t)), "unit": "us/frame", "cores": cores, "kind": "oracle",
            "sample": f"{len(times)} ELT frames (first dropped from the stats) through the FP64 oracle: "
                      f"calibration, CoG, R s with R promoted to float64 once, integrator; mean "
                      f"{t.mean():.0f} us, p99 {np.percentile(t, 99):.0f} us"}


def run_multi(args):
    """Several sensors in one persistent launch: autotuned, timed, and replayed from a graph."""
    import torch
    from aosim.multi import ELT_MULTI, MultiScenario
    from paper_1805_07254_amd import rtc
    from paper_1805_07254_amd.stats import frame_stats, ticks_to_us

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    rtc.load_library()
    t0 = time.time()
    sc = MultiScenario(ELT_MULTI)
    cfg = sc.cfg
    log(f"workload {cfg.name}: {len(cfg.sensors)} sensors, {sum(sc.n_valid)} subapertures, {sc.n_slopes} slopes, "
        f"{sc.n_act} actuators")
    R = sc.control_matrix
    log(f"control matrix {R.shape} built at {time.time() - t0:.0f}s")
    ring = np.stack([sc.frame_set(k, sc.all_turbulence_slopes(k)) for k in range(args.multi_ring)])
    log(f"{args.multi_ring} frame sets of {ring.shape[1]} pixels generated at {time.time() - t0:.0f}s")
    ctx = rtc.rtc_init_multi(sc.sensors, sc.n_act, cm_dtype=args.multi_dtype, gain=cfg.gain, leak=cfg.leak)
    rtc.rtc_load_calib_multi(ctx, sc.dark_set, sc.flat_set, sc.thresholds)
    rtc.rtc_load_cmat(ctx, R)
    khz = rtc.rtc_wall_clock_khz(ctx)
    stream = torch.cuda.current_stream()
    ring16 = torch.from_numpy(ring.view(np.int16)).to("cuda:0")
    n_buf = max(args.warmup + args.multi_steps, 1000)
    frames = ring16[torch.arange(n_buf, device="cuda:0") % args.multi_ring].contiguous().view(torch.uint16)
    launch = min(args.launch_frames, args.multi_steps)
    cmd = torch.empty(max(launch, 1000) * sc.n_act, dtype=torch.float32, device="cuda:0")

    tune = rtc.rtc_autotune(ctx, 64, frames, cmd, stream=stream)
    mode = rtc.rtc_get_frame_mode(ctx)
    best = min((r for r in tune if r["us_per_frame"] > 0), key=lambda r: r["us_per_frame"])
    log(f"autotuned: frame mode {mode}, {best['tuning']}, {best['us_per_frame']:.2f} us/frame over 64 frames")
    balance = None
    if mode == rtc.RTC_FRAMES_PERSISTENT:
        balance = rtc.rtc_balance_rows(ctx, 64, frames, cmd, stream=stream)
        log(f"row split: equal {balance['us_equal']:.2f} us/frame, measured {balance['us_split']:.2f} us/frame, "
            f"kept {balance['kept']}")

    def run(first, n, ts=None):
        done, launches = 0, 0
        while done < n:
            m = min(launch, n - done)
            rtc.rtc_frame_batch(ctx, m, frames[first + done:], cmd, ts=None if ts is None else ts[2 * done:],
                                stream=stream)
            done += m
            launches += 1
        return launches

    run(0, args.warmup)
    torch.cuda.synchronize()
    ts = torch.zeros(2 * args.multi_steps, dtype=torch.int64, device="cuda:0")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t1 = time.perf_counter()
    ev0.record(stream)
    launches = run(args.warmup, args.multi_steps, ts)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    rtc.rtc_sync_check(ctx)
    st = ts.cpu().numpy().reshape(-1, 2)
    period = np.diff(ticks_to_us(st[:, 0] - st[0, 0], khz))
    span = ticks_to_us(st[:, 1] - st[:, 0], khz)
    st_period, st_span = frame_stats(period), frame_stats(span)
    launch_ms = ev0.elapsed_time(ev1) / launches
    log(f"frame period p50 {st_period['p50_us']:.2f} us p99 {st_period['p99_us']:.2f} us, "
        f"{launch_ms:.3f} ms per launch of {launch}")

    # graph replay: one recorded batch of 1000 frames replayed
    gts = torch.zeros(2 * 1000, dtype=torch.int64, device="cuda:0")
    graph = {"recorded": False}
    try:
        rtc.rtc_graph_capture(ctx, 1000, frames, cmd, ts=gts)
        graph["recorded"] = True
    except rtc.RtcError as err:
        graph["error"] = str(err)
    if graph["recorded"]:
        periods = []
        reps = max(1, args.multi_steps // 1000)
        for _ in range(reps):
            rtc.rtc_graph_launch(ctx, stream)
            torch.cuda.synchronize()
            g = gts.cpu().numpy().reshape(-1, 2)
            periods.append(np.diff(ticks_to_us(g[:, 0] - g[0, 0], khz)))
        rtc.rtc_sync_check(ctx)
        graph["replays"] = reps
        graph["frame_period_us"] = frame_stats(np.concatenate(periods))
        log(f"graph replay: frame period p50 {graph['frame_period_us']['p50_us']:.2f} us")
    rtc.rtc_destroy(ctx)

    esz = {"f32": 4, "f16": 2, "bf16": 2, "fp8e4m3": 1}[args.multi_dtype]
    npx = sum(n * s.n_pix * s.n_pix for n, s in zip(sc.n_valid, cfg.sensors))
    fb = sc.n_act * sc.n_slopes * esz + (0 if esz == 4 else 4 * sc.n_act) + npx * 10 + 8 * sc.n_slopes + 8 * sc.n_act
    achieved = fb * launch / (launch_ms * 1e6) if args.multi_steps % launch == 0 else fb / (wall * 1e6 / args.multi_steps) / 1e3
    result = {
        "metric": METRIC, "value": round(st_period["p50_us"], 3), "unit": "us", "n_gpus": 1,
        "steps": args.multi_steps, "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.multi_steps, 6),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": args.multi_dtype,
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: 6 x 74x74 SH (10x10 px) + 3 x 16x16 SH (6x6 px), obscuration 0.28, "
                               f"{sc.n_slopes} slopes, {sc.n_act} actuators on two DMs, "
                               f"{args.multi_dtype} control matrix {sc.n_act * sc.n_slopes * esz / 1e6:.1f} MB",
                   "frames_per_launch": launch, "distinct_frame_sets": args.multi_ring,
                   "frame_mode": "persistent" if mode == 1 else "per-launch", "tuning": best["tuning"],
                   "row_split": balance},
        "frame_period_us": st_period, "frame_span_us": st_span,
        "graph_replay": graph, "autotune": tune,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None, "bytes_per_frame": fb,
                     "kernel": "frames_kernel (persistent, slope panels)" if mode == 1 else
                     "calib_cog_kernel + mvm_panel_kernel (per launch, slope panels)"},
    }
    print(json.dumps(result), flush=True)


def run_pipe(args):
    """Pixel-stream processing at the ELT size: last-pixel -> last-command latency of a camera
    emulated inside the launch, for full-frame processing, pixel-stream processing with equal
    and linearly decreasing subaperture allocation, and with the tail band on every workgroup;
    per-worker end of computation relative to the last pixel; and, for context, the
    whole-frame time of the persistent kernel with the frame already in memory."""
    import torch
    from aosim import ELT, Scenario
    from paper_1805_07254_amd import rtc
    from paper_1805_07254_amd.stats import frame_stats, ticks_to_us

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    rtc.load_library()
    t0 = time.time()
    sc = Scenario(ELT)
    cfg = sc.cfg
    R = sc.control_matrix
    n_ring = 16
    ring = np.stack([sc.frame(k, sc.turbulence_slopes(k)) for k in range(n_ring)])
    log(f"{cfg.name}: matrix and {n_ring} frames at {time.time() - t0:.0f}s")
    ctx = rtc.rtc_init(sc.mask, cfg.n_pix, sc.n_act, gain=cfg.gain, leak=cfg.leak)
    rtc.rtc_load_calib(ctx, sc.dark, sc.flat, cfg.threshold)
    rtc.rtc_load_cmat(ctx, R)
    khz = rtc.rtc_wall_clock_khz(ctx)
    F = args.pipe_frames
    ring16 = torch.from_numpy(ring.reshape(n_ring, -1).view(np.int16)).to("cuda:0")
    frames = ring16[torch.arange(F, device="cuda:0") % n_ring].contiguous().view(torch.uint16)
    cmd = torch.empty(F * sc.n_act, dtype=torch.float32, device="cuda:0")
    skip = min(10, F // 10)

    def mode(name, **kw):
        rtc.rtc_reset(ctx)
        rtc.rtc_pipe_setup(ctx, frame_period_us=args.pipe_period_us, readout_us=args.pipe_readout_us,
                           rows_per_packet=2, **kw)
        info = rtc.rtc_pipe_info(ctx)
        P = info["n_workers"]
        cam = torch.zeros(4 * F, dtype=torch.int64, device="cuda:0")
        wk = torch.zeros(2 * F * P, dtype=torch.int64, device="cuda:0")
        rtc.rtc_pipe_run(ctx, F, frames, cmd, cam_ts=cam, worker_ts=wk)
        torch.cuda.synchronize()
        rtc.rtc_sync_check(ctx)
        cam = cam.cpu().numpy().reshape(F, 4)[skip:]
        wk = wk.cpu().numpy().reshape(F, P, 2)[skip:]
        last = cam[:, 2:3]
        lat = ticks_to_us(wk[:, :, 1].max(axis=1) - cam[:, 2], khz)
        part = ticks_to_us(wk[:, :, 0] - last, khz).mean(axis=0)          # per worker: partial published
        done = ticks_to_us(wk[:, :info["n_owners"], 1] - last, khz).mean(axis=0)   # per owner: rows stored
        st = frame_stats(lat)
        rec = {"mode": name, **kw, "workers": P, "owners": info["n_owners"], "lds_cols": info["lds_cols"],
               "tail_subaps": info["n_tail"],
               "max_subaps_per_worker": info["max_subaps"], "latency_us": st,
               "worker_partial_vs_last_pixel_us": {"last_worker": round(float(part[-1]), 2),
                                                   "max": round(float(part.max()), 2),
                                                   "median": round(float(np.median(part)), 2),
                                                   "profile": [round(float(x), 1) for x in part]},
               "owner_done_vs_last_pixel_us": {"max": round(float(done.max()), 2),
                                                "min": round(float(done.min()), 2)},
               "camera_slip_us": frame_stats(ticks_to_us(cam[:, 3], khz)),
               "readout_us": frame_stats(ticks_to_us(cam[:, 2] - cam[:, 0], khz))}
        log(f"{name}: latency p50 {st['p50_us']:.2f} us p99 {st['p99_us']:.2f} us rms {st['rms_jitter_us']:.2f} us; "
            f"last worker's partial {part[-1]:+.1f} us vs last pixel; camera slip p99 "
            f"{rec['camera_slip_us']['p99_us']:.1f} us")
        return rec

    modes = [mode("full frame, equal allocation", full_frame=True, alloc_ratio=1.0),
             mode("pixel stream, equal allocation", alloc_ratio=1.0),
             mode("pixel stream, linearly decreasing allocation", alloc_ratio=8.0),
             mode("pixel stream, linearly decreasing allocation, tail band on every workgroup", alloc_ratio=8.0,
                  tail_rows=1)]
    sweep = []
    keep = F
    F = min(F, 300)
    for ratio in (2.0, 4.0, 16.0):
        r = mode(f"pixel stream, ratio {ratio:g}", alloc_ratio=ratio)
        sweep.append({"alloc_ratio": ratio, "p50_us": r["latency_us"]["p50_us"], "p99_us": r["latency_us"]["p99_us"]})
    for tail in (2, 3):
        r = mode(f"pixel stream, ratio 8, tail {tail}", alloc_ratio=8.0, tail_rows=tail)
        sweep.append({"alloc_ratio": 8.0, "tail_rows": tail, "p50_us": r["latency_us"]["p50_us"],
                      "p99_us": r["latency_us"]["p99_us"]})
    F = keep

    # whole frame already in memory: the persistent kernel's frame span (start -> last command)
    rtc.rtc_reset(ctx)
    rtc.rtc_set_frame_mode(ctx, rtc.RTC_FRAMES_PERSISTENT)
    ts = torch.zeros(2 * F, dtype=torch.int64, device="cuda:0")
    rtc.rtc_frame_batch(ctx, F, frames, cmd, ts=ts)
    torch.cuda.synchronize()
    rtc.rtc_sync_check(ctx)
    st = ts.cpu().numpy().reshape(F, 2)[skip:]
    whole = frame_stats(ticks_to_us(st[:, 1] - st[:, 0], khz))
    rtc.rtc_destroy(ctx)
    best = modes[-1]["latency_us"]
    result = {
        "metric": "ELT-SCAO last pixel -> DM command latency with pixel-stream processing (us)",
        "value": round(best["p50_us"], 3), "unit": "us", "n_gpus": 1, "steps": args.pipe_frames, "warmup": skip,
        "ms_per_step": args.pipe_period_us / 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {sc.n_valid} subapertures (10x10 px, 740x740 frame), {sc.n_act} "
                               f"actuators, f32 matrix; camera emulated in the launch: {args.pipe_period_us:g} us "
                               f"frame period, rows landing uniformly over {args.pipe_readout_us:g} us, 2-row packets",
                   "distinct_frames": n_ring},
        "p99_us": round(best["p99_us"], 3), "rms_jitter_us": round(best["rms_jitter_us"], 3),
        "modes": modes, "sweep": sweep,
        "whole_frame_in_memory_persistent_span_us": whole,
        "paper_context": {"equal_allocation_latency_ms": 0.84, "unequal_allocation_latency_ms": 0.64,
                          "camera_hz": 500, "hardware": "Xeon Phi KNL + GigE camera"},
        "roofline": None,
    }
    print(json.dumps(result), flush=True)


def run_predict(args):
    """Learned predictor at the ELT size: closed-loop telemetry of the integrator, training with the
    library's kernels, closed-loop judgement against the integrator, and per-frame cost."""
    import torch
    from aosim import ELT, Scenario
    from aosim.telemetry import Telemetry, kl_basis
    from paper_1805_07254_amd import predict, rtc

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    rtc.load_library()
    t0 = time.time()
    dev = torch.device("cuda:0")
    sc = Scenario(ELT)
    cfg = sc.cfg
    ns, na, nm, H = 2 * sc.n_valid, sc.n_act, args.pred_modes, args.pred_history
    D = torch.from_numpy(sc.interaction.astype(np.float32)).to(dev)
    R = sc.control_matrix
    log(f"{cfg.name}: D and R built at {time.time() - t0:.0f}s")
    tel = Telemetry(sc.mask, cfg.pitch, config_index=cfg.index, device=dev)
    seg_len = 2000
    n_train = max(1, args.pred_frames // seg_len)
    ol = torch.cat([tel.segment(k, seg_len)[::8] for k in range(min(n_train, 12))])
    P = kl_basis(ol, nm)                                  # offline preparation on the host
    PD = (P.astype(np.float64) @ sc.interaction.astype(np.float64)).astype(np.float32)
    del ol
    log(f"{nm} KL modes at {time.time() - t0:.0f}s")
    ctx = predict.make_context(sc, R, gain=cfg.gain)
    zs = []
    for seg in range(n_train + 1):                       # last one: validation
        s = tel.segment(seg, seg_len)
        out = predict.run_loop(D, s, tel.noise(seg, seg_len, ns), ctx)
        zs.append(predict.pol_modes(out["residual"], out["cmd_prev"], P, PD))
        if (seg + 1) % 10 == 0:
            log(f"telemetry: {(seg + 1) * seg_len} closed-loop frames at {time.time() - t0:.0f}s")
    mean, std = predict.change_stats(np.concatenate(zs[:n_train]))
    xs, ys = zip(*[predict.windows(z, H, mean, std) for z in zs[:n_train]])
    x, y = predict.to_device(np.concatenate(xs), dev), predict.to_device(np.concatenate(ys), dev)
    del xs, ys
    xv_h, yv_h = predict.windows(zs[n_train], H, mean, std)
    xv, yv = predict.to_device(xv_h, dev), predict.to_device(yv_h, dev)
    net = rtc.MlpNet(H * nm, args.pred_hidden, nm, args.pred_batch)
    net.set_params(*predict.init_params(H * nm, args.pred_hidden, nm, seed=5))
    persist = float(((xv_h[:, -nm:].astype(np.float64) - yv_h) ** 2).mean())   # forecast = the last change again
    t1 = time.time()
    hist = predict.train(net, x, y, epochs=args.pred_epochs, batch=args.pred_batch, lr=1e-3, seed=6, x_val=xv,
                         y_val=yv, log=log)
    train_s = time.time() - t1
    steps = args.pred_epochs * (x.shape[0] // args.pred_batch)

    # one training step's device time (HIP events on the launch stream)
    stream = torch.cuda.current_stream()
    loss = torch.zeros(1, device=dev)
    xb, yb = x[:args.pred_batch].contiguous(), y[:args.pred_batch].contiguous()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(50):
        net.loss_grad(args.pred_batch, xb, yb, loss, stream=stream)
    ev1.record(stream)
    ev1.synchronize()
    step_ms = ev0.elapsed_time(ev1) / 50
    n_in, nh = H * nm, args.pred_hidden
    flops = 2 * args.pred_batch * (2 * n_in * nh + 3 * nh * nm)   # forward 2 products, backward 3
    log(f"training: {steps} steps in {train_s:.1f}s; forward+backward {step_ms:.3f} ms "
        f"({flops / step_ms / 1e9:.1f} TFLOP/s)")

    # judge on held-out segments
    pred = rtc.Predictor(net, H, P, PD, mean, std, cfg.gain)
    judged = []
    for seg in (n_train + 1, n_train + 2):
        s = tel.segment(seg, seg_len)
        nz = tel.noise(seg, seg_len, ns)
        base = predict.run_loop(D, s, nz, ctx)
        withp = predict.run_loop(D, s, nz, ctx, pred)
        judged.append({"segment": seg, "open_loop": predict.residual_rms(s + nz, 100),
                       "integrator": predict.residual_rms(base["residual"], 100),
                       "predictive": predict.residual_rms(withp["residual"], 100)})
        log(f"segment {seg}: {judged[-1]}")

    # per-frame cost on slopes: integrator alone vs predictor step + integrator
    r = torch.zeros((ns + 15) // 16 * 16, device=dev)
    r[:ns] = s[500] + nz[500]
    r2 = torch.empty_like(r)
    c0 = torch.zeros(na, device=dev)
    c1 = torch.empty(na, device=dev)
    st_ptr = stream.cuda_stream

    def timed(fn, reps=2000):
        for _ in range(50):
            fn()
        ev0.record(stream)
        for _ in range(reps):
            fn()
        ev1.record(stream)
        ev1.synchronize()
        return ev0.elapsed_time(ev1) * 1e3 / reps
    t_int = timed(lambda: rtc.rtc_reconstruct_integrate(ctx, r, c1, stream=st_ptr))
    t_pred = timed(lambda: (pred.step(r, c0, r2, stream=st_ptr), rtc.rtc_reconstruct_integrate(ctx, r2, c1,
                                                                                                  stream=st_ptr)))
    t_step = timed(lambda: pred.step(r, c0, r2, stream=st_ptr))

    # frame latency on ELT pixel frames, plain and predictive (device stamps of every frame:
    # first calibration workgroup's start to the last command stored)
    from paper_1805_07254_amd.stats import frame_stats, ticks_to_us
    nfr = args.pred_latency_frames
    ring = np.stack([sc.frame(i, sc.turbulence_slopes(i)) for i in range(16)])
    ring16 = torch.from_numpy(ring.reshape(16, -1).view(np.int16)).to(dev)
    pix = ring16[torch.arange(nfr, device=dev) % 16].contiguous().view(torch.uint16)
    cmdb = torch.empty(nfr * na, device=dev)
    khz = rtc.rtc_wall_clock_khz(ctx)

    def latency(run):
        rtc.rtc_reset(ctx)
        pred.reset()
        ts = torch.zeros(2 * nfr, dtype=torch.int64, device=dev)
        run(ts)
        torch.cuda.synchronize()
        rtc.rtc_sync_check(ctx)
        t = ts.cpu().numpy().reshape(-1, 2)
        return {"frame_span_us": frame_stats(ticks_to_us(t[:, 1] - t[:, 0], khz), skip=100),
                "frame_period_us": frame_stats(np.diff(ticks_to_us(t[:, 0] - t[0, 0], khz)), skip=100)}
    lat = {"frames": nfr, "skip": 100,
           "integrator_per_launch": latency(lambda ts: rtc.rtc_frame_batch(ctx, nfr, pix, cmdb, ts=ts, stream=stream)),
           "predictive_per_launch": latency(lambda ts: pred.frame_batch(ctx, nfr, pix, cmdb, ts=ts, stream=stream))}
    rtc.rtc_set_frame_mode(ctx, rtc.RTC_FRAMES_PERSISTENT)
    lat["integrator_persistent"] = latency(lambda ts: rtc.rtc_frame_batch(ctx, nfr, pix, cmdb, ts=ts, stream=stream))
    # the predictive frames in one persistent launch (the step's four phases between grid barriers)
    lat["predictive_persistent"] = latency(lambda ts: pred.frame_batch(ctx, nfr, pix, cmdb, ts=ts, stream=stream))
    lat["predictive_persistent_ran"] = ("persistent" if pred.last_batch_mode() == rtc.RTC_FRAMES_PERSISTENT
                                        else "per launch (shape not built)")
    log("frame span p50/p99 (us): " + ", ".join(
        f"{k} {v['frame_span_us']['p50_us']:.2f}/{v['frame_span_us']['p99_us']:.2f}"
        for k, v in lat.items() if isinstance(v, dict)))
    pred.close()
    net.close()
    rtc.rtc_destroy(ctx)
    res_i = float(np.mean([j["integrator"] for j in judged]))
    res_p = float(np.mean([j["predictive"] for j in judged]))
    result = {
        "metric": "closed-loop residual slope RMS, learned predictor vs integrator (px)",
        "value": round(res_p, 5), "unit": "px", "n_gpus": 1, "steps": steps, "warmup": 0,
        "ms_per_step": round(step_ms, 4), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {sc.n_valid} subapertures, {na} actuators, two frozen-flow layers "
                               f"(8 and 20 m/s, 1 kHz, 0.05 px noise), {nm} KL modes, network "
                               f"{H}x{nm} -> {args.pred_hidden} (GELU) -> {nm}, {n_train * seg_len} training frames",
                   "epochs": args.pred_epochs, "batch": args.pred_batch},
        "integrator_residual_px": round(res_i, 5), "predictive_residual_px": round(res_p, 5),
        "gain_percent": round(100 * (1 - res_p / res_i), 2), "judged_segments": judged,
        "validation_mse": {"last_change": persist, "zero_change": float((yv_h.astype(np.float64) ** 2).mean()),
                           "trained": hist[-1].get("val_loss")}, "training": hist,
        "frame_cost_us": {"integrator": round(t_int, 3), "predictor_step_plus_integrator": round(t_pred, 3),
                          "predictor_step": round(t_step, 3),
                          "note": "HIP events over back-to-back calls on slopes (host-enqueued)"},
        "frame_latency": lat,
        "training_step": {"ms": round(step_ms, 4), "tflops": round(flops / step_ms / 1e9, 2),
                          "peak_bf16_tflops": 2500.0},
    }
    print(json.dumps(result), flush=True)


def cpu_single_core(seconds: float) -> dict:
    """CPU leg on one core, in a child process pinned to one core of this
    process's affinity set with one BLAS thread."""
    import subprocess
    core = sorted(os.sched_getaffinity(0))[0]
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "BLIS_NUM_THREADS"):
        env[k] = "1"
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-leg", str(core), "--cpu-seconds", str(seconds)]
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=seconds * 4 + 300)
    if r.returncode != 0:
        return {"error": f"child exited {r.returncode}: {r.stderr[-400:]}"}
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_leg_child(core: int, seconds: float) -> None:
    """Entry of the single-core child: pin, rebuild the workload, time the oracle."""
    os.sched_setaffinity(0, {core})
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:                                          # the environment already asks for one thread
        pass
    from aosim import ELT, Scenario
    sc = Scenario(ELT)
    ring = np.stack([sc.frame(i, sc.turbulence_slopes(i)) for i in range(8)])
    out = cpu_baseline(sc, ring, seconds)
    out["cores"] = len(os.sched_getaffinity(0))
    out["sample"] = "one core, one BLAS thread, separate process: " + out["sample"]
    print(json.dumps(out), flush=True)


def stage_breakdown(tr: np.ndarray, khz: int) -> dict:
    """Per-frame critical path of traced persistent frames: [frames, groups, 8]
    stamps (frame start, slopes issued, barrier passed, slices loaded, sums
    done, commands written, stores complete, arrival counted)."""
    from paper_1805_07254_amd.stats import ticks_to_us
    t = tr.astype(np.int64)
    start = t[:, :, 0].min(axis=1)
    last_arrival = t[:, :, 7].max(axis=1)
    first_arrival = t[:, :, 7].min(axis=1)
    last_pass = t[:, :, 2].max(axis=1)
    last_cmd = t[:, :, 5].max(axis=1)
    us = lambda d: ticks_to_us(d, khz)
    med = lambda x: round(float(np.median(x)), 3)
    return {
        "frames": int(t.shape[0]), "groups": int(t.shape[1]),
        "start_to_last_arrival_us": med(us(last_arrival - start)),
        "arrival_spread_us": med(us(last_arrival - first_arrival)),
        "barrier_us": med(us(last_pass - last_arrival)),
        "barrier_to_last_commands_us": med(us(last_cmd - last_pass)),
        "calibration_us": med(us(np.median(t[:, :, 1] - t[:, :, 0], axis=1))),
        "slice_load_us": med(us(np.median(t[:, :, 3] - t[:, :, 2], axis=1))),
        "partial_sums_us": med(us(np.median(t[:, :, 4] - t[:, :, 3], axis=1))),
        "span_us": med(us(last_cmd - start)),
    }


def load_counters(frames_per_launch: int):
    """rocprofv3 counters of the frames kernel from the committed profile, when
    it was taken on the current kernel sources at the same frames per launch."""
    if not os.path.exists(PROFILE_COUNTERS):
        return None, "no counter profile"
    try:
        prof = json.load(open(PROFILE_COUNTERS))
    except Exception as err:                                  # unreadable profile: report, do not use
        return None, f"counter profile unreadable: {err}"
    if prof.get("kernel_source_sha256_16") != kernel_source_hash():
        return None, "counter profile taken on other kernel sources"
    if prof.get("frames_per_launch") != frames_per_launch:
        return None, f"counter profile taken at {prof.get('frames_per_launch')} frames per launch"
    return prof, None


def frame_model(prof: dict, frames: int, frame_us: float, barrier_us: float) -> dict:
    """Floor of the persistent frame from its counted work: the measured barrier
    latency plus the largest of the VALU-issue, LDS, L2 and HBM times of one
    frame (per compute unit where the resource is per unit)."""
    c = prof["counters_per_dispatch"]
    per_cu = lambda v: v / frames / N_CU
    clk = CLK_GHZ * 1e3                                        # cycles per us
    t_valu = per_cu(c["SQ_INSTS_VALU"]) / clk                  # one wave64 VALU instruction per cycle per CU
    lds_bytes = c["SQ_INSTS_LDS_LOAD_BANDWIDTH"] * 64
    t_lds = per_cu(lds_bytes) / LDS_BYTES_PER_CLK / clk
    l2_bytes = c["TCP_TCC_READ_REQ_sum"] * TCP_REQ_BYTES
    t_l2 = per_cu(l2_bytes) / L2_BYTES_PER_CLK_PER_CU / clk
    hbm_bytes = prof.get("hbm_bytes_per_dispatch")
    t_hbm = hbm_bytes / frames / (HBM_PEAK_GBPS * 1e3) if hbm_bytes else 0.0
    terms = {"valu_issue_us": t_valu, "lds_us": t_lds, "l2_us": t_l2, "hbm_us": t_hbm}
    floor = barrier_us + max(terms.values())
    return {
        "terms_us": {k: round(v, 4) for k, v in terms.items()},
        "barrier_floor_us": round(barrier_us, 4),
        "floor_us": round(floor, 4), "frame_us": round(frame_us, 4), "frac": round(floor / frame_us, 4),
        "per_frame": {"valu_insts": round(c["SQ_INSTS_VALU"] / frames), "fma_f32_insts": round(
            c["SQ_INSTS_VALU_FMA_F32"] / frames), "lds_load_bytes": round(lds_bytes / frames),
            "l2_read_bytes": round(l2_bytes / frames)},
        "source": os.path.relpath(PROFILE_COUNTERS, ROOT),
    }


def main():
    args = parse()
    if args.cpu_leg is not None:
        cpu_leg_child(args.cpu_leg, args.cpu_seconds)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    run = {"elt-multi": run_multi, "elt-predict": run_predict, "elt-pipe": run_pipe}.get(args.workload, run_scao)
    run(args)
    # explicit teardown: every context is closed, the device is idle, and the
    # library's HIP modules are unregistered now rather than from the exit
    # handlers, after a profiler attached to the process has finalised
    import gc
    import torch
    from paper_1805_07254_amd import rtc
    gc.collect()
    torch.cuda.synchronize()
    rtc.unload_library()


def run_scao(args):
    import torch
    from aosim import ELT, Scenario
    from paper_1805_07254_amd import rtc
    from paper_1805_07254_amd.stats import frame_stats, ticks_to_us

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    rtc.load_library()
    t_setup = time.time()
    sc = Scenario(ELT)
    cfg = sc.cfg
    log(f"workload {cfg.name}: {sc.n_valid} subapertures, {2 * sc.n_valid} slopes, {sc.n_act} actuators")
    R = sc.control_matrix
    log(f"control matrix {R.shape} built ({R.nbytes / 1e6:.1f} MB) at {time.time() - t_setup:.0f}s")
    ring = np.empty((args.ring, cfg.frame_side, cfg.frame_side), np.uint16)
    for i in range(args.ring):
        ring[i] = sc.frame(i, sc.turbulence_slopes(i))
        if (i + 1) % 32 == 0:
            log(f"generated {i + 1}/{args.ring} open-loop frames")
    log(f"setup done in {time.time() - t_setup:.0f}s")

    n_act = sc.n_act
    ring16 = torch.from_numpy(ring.reshape(args.ring, -1).view(np.int16)).to("cuda:0")
    dev_ring = ring16.view(torch.uint16)
    n_buf = max(args.warmup + args.steps, 200 + args.variant_steps, args.roofline_frames, args.paced_frames,
                200 + args.horizontal_steps, args.trace_frames)
    frames = ring16[torch.arange(n_buf, device="cuda:0") % args.ring].contiguous().view(torch.uint16)
    log(f"frame buffer: {n_buf} frames, {frames.numel() * 2 / 1e9:.2f} GB on the device")
    cmd = torch.empty(max(args.launch_frames, args.roofline_frames, args.paced_frames) * n_act,
                      dtype=torch.float32, device="cuda:0")
    stream = torch.cuda.current_stream()
    tuning = dict(kernel=args.mvm_kernel, k_split=args.k_split, rows_per_wave=args.rows_per_wave,
                  unroll=args.unroll, blocks=args.blocks, waves=args.waves)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count

    def make_ctx(fmt, mode):
        ctx = rtc.rtc_init(sc.mask, cfg.n_pix, n_act, cm_dtype=fmt, gain=cfg.gain, leak=cfg.leak)
        rtc.rtc_load_calib(ctx, sc.dark, sc.flat, cfg.threshold)
        rtc.rtc_load_cmat(ctx, R)
        rtc.rtc_set_mvm_tuning(ctx, **(tuning if fmt == "f32" else {k: v for k, v in tuning.items()
                                                                       if k != "kernel"}))
        rtc.rtc_set_frame_mode(ctx, mode)
        return ctx

    def run(ctx, first, n, per_launch, ts=None):
        """Frames [first, first + n) of the buffer, per_launch per launch; returns launches."""
        done, launches = 0, 0
        while done < n:
            m = min(per_launch, n - done)
            rtc.rtc_frame_batch(ctx, m, frames[first + done:], cmd, ts=None if ts is None else ts[2 * done:],
                                stream=stream)
            done += m
            launches += 1
        return launches

    def series(ts, khz):
        st = ts.cpu().numpy().reshape(-1, 2)
        start_us = ticks_to_us(st[:, 0] - st[0, 0], khz)
        end_us = ticks_to_us(st[:, 1] - st[0, 0], khz)
        return np.diff(start_us), end_us - start_us

    def timed(ctx, warm, n, khz, per_launch):
        run(ctx, 0, warm, per_launch)
        torch.cuda.synchronize()
        ts = torch.zeros(2 * n, dtype=torch.int64, device="cuda:0")
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        launches = run(ctx, warm, n, per_launch, ts)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        rtc.rtc_sync_check(ctx)
        period, span = series(ts, khz)
        inside = np.ones(len(period), bool)                   # periods that do not straddle a relaunch
        inside[per_launch - 1::per_launch] = False
        return {"period": period, "period_inside": period[inside], "span": span, "wall": wall,
                "launch_ms": ev0.elapsed_time(ev1) / launches, "launches": launches}

    # --- headline: FP32 matrix, persistent kernel; the timed steps
    ctx = make_ctx("f32", rtc.RTC_FRAMES_PERSISTENT)
    khz = rtc.rtc_wall_clock_khz(ctx)
    balance = None
    if args.balance_rows:
        balance = rtc.rtc_balance_rows(ctx, min(256, args.launch_frames), frames, cmd, stream=stream)
        log(f"row split: equal {balance['us_equal']:.2f} us/frame, measured {balance['us_split']:.2f} us/frame, "
            f"kept {balance['kept']}")
    log(f"warm-up {args.warmup} frames, then {args.steps} timed frames (persistent, "
        f"{args.launch_frames} per launch)")
    head = timed(ctx, args.warmup, args.steps, khz, args.launch_frames)
    st_span = frame_stats(head["span"])
    st_period = frame_stats(head["period"]) if len(head["period"]) else None
    log(f"timed frames: span p50 {st_span['p50_us']:.2f} us p99 {st_span['p99_us']:.2f} us, wall "
        f"{head['wall'] * 1e6 / args.steps:.2f} us/frame")

    # --- long runs: whole launches of roofline_frames frames, HIP events on the launch stream.
    # The roofline's device time comes from launches without time stamps (the frame as it runs
    # in production: the stamps' end-of-frame reduction costs a workgroup a memory round trip);
    # the latency distribution from launches with them.
    def whole_launch(ts):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        rtc.rtc_frame_batch(ctx, args.roofline_frames, frames, cmd, ts=ts, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1)
    launch_ms = [whole_launch(None) for _ in range(args.roofline_launches)]
    long_period, long_span, stamped_ms = [], [], []
    for r in range(args.stats_launches):
        ts = torch.zeros(2 * args.roofline_frames, dtype=torch.int64, device="cuda:0")
        stamped_ms.append(whole_launch(ts))
        pr, sp = series(ts, khz)
        long_period.append(pr)
        long_span.append(sp)
    rtc.rtc_sync_check(ctx)
    launch_avg_ms = float(np.mean(launch_ms))
    frame_us = launch_avg_ms * 1e3 / args.roofline_frames
    long_run = {"frames_per_launch": args.roofline_frames,
                "launches_without_stamps_ms": [round(x, 4) for x in launch_ms],
                "launches_with_stamps_ms": [round(x, 4) for x in stamped_ms]}
    if long_period:
        lp, ls = np.concatenate(long_period), np.concatenate(long_span)
        long_run.update({
            "frame_period_us": frame_stats(lp), "frame_span_us": frame_stats(ls),
            "frame_period_us_skip100": frame_stats(long_period[0], skip=100) if len(long_period[0]) > 200
            else None,
            "frame_span_us_skip100": frame_stats(long_span[0], skip=100) if len(long_span[0]) > 200 else None})
    log(f"{args.roofline_launches} launches of {args.roofline_frames} frames without stamps: {launch_avg_ms:.3f} ms "
        f"each ({frame_us:.3f} us/frame); with stamps: "
        f"{np.mean(stamped_ms) * 1e3 / args.roofline_frames if stamped_ms else float('nan'):.3f} us/frame" +
        (f", span p50 {long_run['frame_span_us']['p50_us']:.2f} us, p99 {long_run['frame_span_us']['p99_us']:.2f} us"
         if long_period else ""))

    # --- stage trace of every workgroup: the measured barrier floor
    G = min(n_cu if args.blocks <= 0 else args.blocks, n_act)
    trace = torch.zeros(args.trace_frames * G * 8, dtype=torch.int64, device="cuda:0")
    rtc.rtc_set_trace(ctx, trace, args.trace_frames, G)
    rtc.rtc_frame_batch(ctx, args.trace_frames, frames, cmd, stream=stream)
    torch.cuda.synchronize()
    rtc.rtc_set_trace(ctx)
    rtc.rtc_sync_check(ctx)
    stages = stage_breakdown(trace.cpu().numpy().reshape(args.trace_frames, G, 8)[min(100, args.trace_frames // 2):],
                             khz)
    del trace
    log(f"stages (median per frame): {stages}")

    # --- host-paced frames: released at a fixed period through a host word
    paced = None
    if args.paced_frames > 0:
        ts = torch.zeros(2 * args.paced_frames, dtype=torch.int64, device="cuda:0")
        log(f"host-paced: {args.paced_frames} frames every {args.paced_period_us} us")
        rel, done = rtc.rtc_paced_batch(ctx, args.paced_frames, frames, cmd, args.paced_period_us, ts=ts,
                                        stream=stream)
        rtc.rtc_sync_check(ctx)
        host_lat = (done - rel) / 1e3
        late = (rel - np.arange(args.paced_frames) * args.paced_period_us * 1e3) / 1e3
        _, pspan = series(ts, khz)
        paced = {"frames": args.paced_frames, "period_us": args.paced_period_us,
                 "host_latency_us": frame_stats(host_lat),
                 "host_latency_us_skip100": frame_stats(host_lat, skip=100) if args.paced_frames > 200 else None,
                 "device_span_us": frame_stats(pspan),
                 "device_span_us_skip100": frame_stats(pspan, skip=100) if args.paced_frames > 200 else None,
                 "release_lateness_us": frame_stats(late),
                 "note": "host latency = release word written -> done word seen by the releasing thread; "
                         "device span = first workgroup's frame start -> last command store"}
        log(f"host-paced latency p50 {paced['host_latency_us']['p50_us']:.2f} us p99 "
            f"{paced['host_latency_us']['p99_us']:.2f} us, device span p50 "
            f"{paced['device_span_us']['p50_us']:.2f} us")
    rtc.rtc_destroy(ctx)

    # --- horizontal split (the paper's processing strategy), same frames
    horizontal = None
    if args.horizontal_steps > 0:
        try:
            hctx = make_ctx("f32", rtc.RTC_FRAMES_HORIZONTAL)
        except rtc.RtcError as err:
            horizontal = {"error": str(err)}
        else:
            h = timed(hctx, 200, args.horizontal_steps, khz, args.launch_frames)
            horizontal = {"frame_period_us": frame_stats(h["period"]), "frame_span_us": frame_stats(h["span"]),
                          "launch_ms": round(h["launch_ms"], 4)}
            rtc.rtc_destroy(hctx)
            log(f"horizontal split: span p50 {horizontal['frame_span_us']['p50_us']:.2f} us")

    # --- per-launch mode (calibration kernel + reconstruction kernel per frame)
    ctx = make_ctx("f32", rtc.RTC_FRAMES_PER_LAUNCH)
    pl = timed(ctx, 200, args.variant_steps, khz, args.launch_frames)
    per_launch = {"frame_period_us": frame_stats(pl["period"]), "frame_span_us": frame_stats(pl["span"])}
    log(f"per-launch frames: span p50 {per_launch['frame_span_us']['p50_us']:.2f} us")

    # the two kernels of the per-launch mode alone, HIP events on the launch stream
    slopes = torch.empty(2 * sc.n_valid, dtype=torch.float32, device="cuda:0")
    rtc.rtc_calibrate_centroid(ctx, dev_ring[0], slopes, stream=stream)
    out_cmd = torch.empty(n_act, dtype=torch.float32, device="cuda:0")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s_ptr, c_ptr, st_ptr = slopes.data_ptr(), out_cmd.data_ptr(), stream.cuda_stream
    frame_ptrs = [dev_ring[i].data_ptr() for i in range(args.ring)]

    def kernel_us(fn, reps):
        for _ in range(min(50, reps)):
            fn(0)
        ev0.record(stream)
        for i in range(reps):
            fn(i)
        ev1.record(stream)
        ev1.synchronize()
        return ev0.elapsed_time(ev1) * 1e3 / reps

    mvm_us = kernel_us(lambda i: rtc.rtc_reconstruct_integrate(ctx, s_ptr, c_ptr, stream=st_ptr), args.kernel_reps)
    cal_us = kernel_us(lambda i: rtc.rtc_calibrate_centroid(ctx, frame_ptrs[i % args.ring], s_ptr, stream=st_ptr),
                       args.kernel_reps)
    ldr = (2 * sc.n_valid + 3) // 4 * 4
    mvm_bytes = n_act * ldr * 4 + ldr * 4 + 3 * n_act * 4        # R, s, state r/w, cmd w
    log(f"reconstruct+integrate {mvm_us:.2f} us/launch ({mvm_bytes / mvm_us / 1e3:.0f} GB/s), "
        f"calibrate+centroid {cal_us:.2f} us/launch")
    rtc.rtc_destroy(ctx)

    # --- read-bandwidth probes over working sets from inside the Infinity Cache to far beyond it,
    # and a plain copy (the traffic counters' calibration kernel)
    probes = {}
    pctx = make_ctx("f32", rtc.RTC_FRAMES_PER_LAUNCH)
    out1 = torch.zeros(1, dtype=torch.float32, device="cuda:0")
    for label in [x for x in args.probes.split(",") if x and x != "none"]:
        nbytes = int(float(label.rstrip("MB")) * 1e6) // 16 * 16 if label.endswith("MB") else \
            int(float(label.rstrip("GB")) * (1 << 30)) // 16 * 16
        buf = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
        reps = 200 if nbytes < (1 << 30) else 20
        us = kernel_us(lambda i: rtc.rtc_probe_read(pctx, buf, nbytes, out1, stream=stream), reps)
        probes[label] = round(nbytes / us / 1e3, 1)
        del buf
    copy_bytes = 256 << 20
    src = torch.empty(copy_bytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    us = kernel_us(lambda i: rtc.rtc_probe_copy(pctx, src, dst, copy_bytes, stream=stream), 10)
    probes["copy_256MiB"] = round(2 * copy_bytes / us / 1e3, 1)
    del src, dst
    rtc.rtc_destroy(pctx)
    log(f"read/copy probes GB/s: {probes}")

    # --- reduced-precision control matrices, persistent kernel, same frames
    variants = {}
    for fmt in [v for v in args.variants.split(",") if v and v != "none"]:
        vctx = make_ctx(fmt, rtc.RTC_FRAMES_PERSISTENT)
        v = timed(vctx, 200, args.variant_steps, khz, args.launch_frames)
        vp, vs = frame_stats(v["period"]), frame_stats(v["span"])
        variants[fmt] = {"frame_span_p50_us": round(vs["p50_us"], 3), "frame_span_p99_us": round(vs["p99_us"], 3),
                         "frame_period_p50_us": round(vp["p50_us"], 3), "frame_period_p99_us": round(vp["p99_us"], 3),
                         "rms_jitter_us": round(vp["rms_jitter_us"], 3),
                         "matrix_MB": round(n_act * 2 * sc.n_valid * FMT_BYTES[fmt] / 1e6, 2),
                         "flops_per_frame": frame_flops(sc)}
        rtc.rtc_destroy(vctx)
        log(f"{fmt}: frame span p50 {vs['p50_us']:.2f} us, period p50 {vp['p50_us']:.2f} us")

    # --- roofline of the frames kernel
    flops = frame_flops(sc)
    fb = frame_bytes(sc, "f32")
    achieved = flops * args.roofline_frames / (launch_avg_ms * 1e-3) / 1e12
    prof, why = load_counters(args.roofline_frames)
    traffic = prof.get("hbm_bytes_per_dispatch") if prof else None
    model = frame_model(prof, args.roofline_frames, frame_us, stages["barrier_us"]) if prof else {"unavailable": why}
    hbm_gbps = fb / frame_us / 1e3
    roofline = {
        "bound": "alu", "achieved": round(achieved, 3), "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
        "frac": round(achieved / VALU_PEAK_TFLOPS, 4), "traffic": traffic,
        "kernel": "frames_kernel (persistent FP32: calibrate, CoG, R s, integrate; slab on chip)",
        "flops_per_frame": flops, "frames_per_launch": args.roofline_frames,
        "launch_ms": round(launch_avg_ms, 4), "frame_us": round(frame_us, 4),
        "model": model,
        "hbm": {"algorithmic_bytes_per_frame": fb, "algorithmic_GBps": round(hbm_gbps, 1),
                "frac_of_peak": round(hbm_gbps / HBM_PEAK_GBPS, 4),
                "frac_of_probes": {k: round(hbm_gbps / v, 4) for k, v in probes.items() if k != "copy_256MiB"},
                "traffic_bytes_per_frame": round(traffic / args.roofline_frames) if traffic else None,
                "note": "the slab stays on chip across frames, so HBM traffic is far below the algorithmic bytes; "
                        "algorithmic GB/s above the HBM peak are the matrix read from registers, LDS and L2"},
    }
    if not prof:
        log(f"roofline model: {why}")

    wall_us = head["wall"] * 1e6 / args.steps
    result = {
        "metric": METRIC,
        "value": round(st_span["p50_us"], 3),
        "unit": "us",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall_us / 1e3, 6),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{cfg.name}: {cfg.n_sub}x{cfg.n_sub} SH, {cfg.n_pix}x{cfg.n_pix} px, "
                        f"obscuration {cfg.obscuration}, {sc.n_valid} subapertures, {2 * sc.n_valid} slopes, "
                        f"{sc.n_act} actuators, FP32 control matrix {R.nbytes / 1e6:.1f} MB",
            "frame_mode": "persistent",
            "row_split": balance,
            "frames_per_launch": args.launch_frames,
            "distinct_frames": args.ring,
            "frame_data": "open-loop frozen-flow von Karman frames (r0 0.15 m, L0 25 m, 10 m/s)",
        },
        "value_is": "p50 of the timed frames' span: first workgroup's frame start to the last workgroup's "
                    "command store (device wall clock)",
        "frame_span_us": st_span,
        "frame_period_us": st_period,
        "frame_period_us_within_launches": frame_stats(head["period_inside"]) if len(head["period_inside"]) else None,
        "long_run": long_run,
        "stages_us": stages,
        "host_paced": paced,
        "horizontal_mode": horizontal,
        "per_launch_mode": per_launch,
        "kernels_us": {"reconstruct_integrate": round(mvm_us, 3), "calibrate_centroid": round(cal_us, 3)},
        "per_launch_gemv_GBps": round(mvm_bytes / mvm_us / 1e3, 1),
        "read_probe_GBps": probes,
        "precision_variants": variants,
        "roofline": roofline,
    }
    if not args.no_cpu:
        log(f"timing the FP64 oracle for ~{args.cpu_seconds:.0f}s on the host (all cores)")
        result["cpu_baseline"] = cpu_baseline(sc, ring, args.cpu_seconds)
        log(f"timing the FP64 oracle for ~{args.cpu_seconds:.0f}s on one core (child process)")
        result["cpu_baseline"]["single_core"] = cpu_single_core(args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
