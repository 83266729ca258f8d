"""Benchmark of the AO real-time-control frame on one MI355X.

One step = one ELT-scale SCAO frame through the whole hot path (calibration,
centre of gravity, control-matrix x slopes, integrator).  Frames run back to
back, as the paper's no-camera measurements do, from a device buffer holding
one raw frame per step (copies of a ring of distinct open-loop frames), so
every frame's pixels are read from HBM.  The headline runs the persistent
kernel, one cooperative launch per --launch-frames frames; the per-frame device
time stamps give the frame time series (start of frame k to start of frame
k+1) whose p50 is ``value``, plus p99, RMS and peak-to-peak jitter, and the
span of each frame (its start to the last workgroup's command store).  The
per-launch mode (two kernels per frame) and the reduced-precision matrix
formats are timed the same way.  The roofline figure divides the algorithmic
bytes of a launch by the launch's average duration from HIP events on the
launch stream, and the FP64 oracle is timed on the host cores as a CPU
baseline.

    python bench.py [--steps 10000] [--warmup 500] [--launch-frames 1000]
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
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "frames_elt_traffic.json")
KERNEL_SRCS = [os.path.join(ROOT, "paper_1805_07254_amd", "csrc", f) for f in ("rtc_kernels.hip", "rtc_device.h")]
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
                   help="reduced-precision matrix formats also timed (comma list, empty = none)")
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
    return {"value": float(np.median(t)), "unit": "us/frame", "cores": int(blas_threads), "kind": "oracle",
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
    P = kl_basis(ol, nm).to(dev)
    PD = P @ D
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
    mean, std = predict.change_stats(torch.cat(zs[:n_train]))
    xs, ys = zip(*[predict.windows(z, H, mean, std) for z in zs[:n_train]])
    x, y = torch.cat(xs), torch.cat(ys)
    del xs, ys
    xv, yv = predict.windows(zs[n_train], H, mean, std)
    net = rtc.MlpNet(H * nm, args.pred_hidden, nm, args.pred_batch)
    net.set_params(*predict.init_params(H * nm, args.pred_hidden, nm, seed=5))
    persist = float(((xv[:, -nm:] - yv) ** 2).mean().item())     # forecast = the last change again
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
    pred = rtc.Predictor(net, H, P.cpu().numpy(), PD.cpu().numpy(), mean.cpu().numpy(), std.cpu().numpy(), cfg.gain)
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
    pred.close()
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
        "validation_mse": {"last_change": persist, "zero_change": float((yv ** 2).mean().item()),
                           "trained": hist[-1].get("val_loss")}, "training": hist,
        "frame_cost_us": {"integrator": round(t_int, 3), "predictor_step_plus_integrator": round(t_pred, 3)},
        "training_step": {"ms": round(step_ms, 4), "tflops": round(flops / step_ms / 1e9, 2),
                          "peak_bf16_tflops": 2500.0},
    }
    print(json.dumps(result), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "elt-multi":
        run_multi(args)
        return
    if args.workload == "elt-predict":
        run_predict(args)
        return
    if args.workload == "elt-pipe":
        run_pipe(args)
        return
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

    npx = cfg.frame_side * cfg.frame_side
    n_act = sc.n_act
    ring16 = torch.from_numpy(ring.reshape(args.ring, -1).view(np.int16)).to("cuda:0")
    dev_ring = ring16.view(torch.uint16)
    n_buf = max(args.warmup + args.steps, 200 + args.variant_steps, args.launch_frames)
    frames = ring16[torch.arange(n_buf, device="cuda:0") % args.ring].contiguous().view(torch.uint16)
    log(f"frame buffer: {n_buf} frames, {frames.numel() * 2 / 1e9:.2f} GB on the device")
    cmd = torch.empty(args.launch_frames * n_act, dtype=torch.float32, device="cuda:0")
    stream = torch.cuda.current_stream()
    tuning = dict(kernel=args.mvm_kernel, k_split=args.k_split, rows_per_wave=args.rows_per_wave,
                  unroll=args.unroll, blocks=args.blocks, waves=args.waves)

    def make_ctx(fmt, mode):
        ctx = rtc.rtc_init(sc.mask, cfg.n_pix, n_act, cm_dtype=fmt, gain=cfg.gain, leak=cfg.leak)
        rtc.rtc_load_calib(ctx, sc.dark, sc.flat, cfg.threshold)
        rtc.rtc_load_cmat(ctx, R)
        rtc.rtc_set_mvm_tuning(ctx, **(tuning if fmt == "f32" else {k: v for k, v in tuning.items()
                                                                       if k != "kernel"}))
        rtc.rtc_set_frame_mode(ctx, mode)
        return ctx

    def run(ctx, first, n, ts=None):
        """Frames [first, first + n) of the buffer, launch_frames per launch; returns launches."""
        done, launches = 0, 0
        while done < n:
            m = min(args.launch_frames, n - done)
            rtc.rtc_frame_batch(ctx, m, frames[first + done:], cmd, ts=None if ts is None else ts[2 * done:],
                                stream=stream)
            done += m
            launches += 1
        return launches

    def timed(ctx, warm, n, khz):
        run(ctx, 0, warm)
        torch.cuda.synchronize()
        ts = torch.zeros(2 * n, dtype=torch.int64, device="cuda:0")
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        launches = run(ctx, warm, n, ts)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        rtc.rtc_sync_check(ctx)
        st = ts.cpu().numpy().reshape(-1, 2)
        start_us = ticks_to_us(st[:, 0] - st[0, 0], khz)
        end_us = ticks_to_us(st[:, 1] - st[0, 0], khz)
        period = np.diff(start_us)
        inside = np.ones(len(period), bool)                   # periods that do not straddle a relaunch
        inside[args.launch_frames - 1::args.launch_frames] = False
        return {"period": period, "period_inside": period[inside], "span": end_us - start_us, "wall": wall,
                "launch_ms": ev0.elapsed_time(ev1) / launches, "launches": launches}

    # --- headline: FP32 matrix, persistent kernel
    ctx = make_ctx("f32", rtc.RTC_FRAMES_PERSISTENT)
    khz = rtc.rtc_wall_clock_khz(ctx)
    balance = None
    if args.balance_rows:
        balance = rtc.rtc_balance_rows(ctx, min(256, args.launch_frames), frames, cmd, stream=stream)
        log(f"row split: equal {balance['us_equal']:.2f} us/frame, measured {balance['us_split']:.2f} us/frame, "
            f"kept {balance['kept']}")
    log(f"warm-up {args.warmup} frames, then {args.steps} timed frames (persistent, "
        f"{args.launch_frames} per launch)")
    head = timed(ctx, args.warmup, args.steps, khz)
    st_period = frame_stats(head["period"])
    st_span = frame_stats(head["span"])
    log(f"frame period p50 {st_period['p50_us']:.2f} us p99 {st_period['p99_us']:.2f} us, span p50 "
        f"{st_span['p50_us']:.2f} us, wall {head['wall'] * 1e6 / args.steps:.2f} us/frame, "
        f"{head['launch_ms']:.3f} ms per launch")
    rtc.rtc_destroy(ctx)

    # --- per-launch mode (calibration kernel + reconstruction kernel per frame)
    ctx = make_ctx("f32", rtc.RTC_FRAMES_PER_LAUNCH)
    pl = timed(ctx, 200, args.variant_steps, khz)
    per_launch = {"frame_period_us": frame_stats(pl["period"]), "frame_span_us": frame_stats(pl["span"])}
    log(f"per-launch frames: period p50 {per_launch['frame_period_us']['p50_us']:.2f} us")

    # the two kernels of the per-launch mode alone, HIP events on the launch stream
    slopes = torch.empty(2 * sc.n_valid, dtype=torch.float32, device="cuda:0")
    rtc.rtc_calibrate_centroid(ctx, dev_ring[0], slopes, stream=stream)
    out_cmd = torch.empty(n_act, dtype=torch.float32, device="cuda:0")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s_ptr, c_ptr, st_ptr = slopes.data_ptr(), out_cmd.data_ptr(), stream.cuda_stream
    frame_ptrs = [dev_ring[i].data_ptr() for i in range(args.ring)]

    def kernel_us(fn, reps):
        for _ in range(50):
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

    # --- read-bandwidth probes at the matrix's working-set size and at 2 GB, and a plain copy
    probes = {}
    pctx = make_ctx("f32", rtc.RTC_FRAMES_PER_LAUNCH)
    out1 = torch.zeros(1, dtype=torch.float32, device="cuda:0")
    for label, nbytes in (("140MB", mvm_bytes // 16 * 16), ("2GB", 2 << 30)):
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
    for fmt in [v for v in args.variants.split(",") if v]:
        vctx = make_ctx(fmt, rtc.RTC_FRAMES_PERSISTENT)
        v = timed(vctx, 200, args.variant_steps, khz)
        vp, vs = frame_stats(v["period"]), frame_stats(v["span"])
        vb = frame_bytes(sc, fmt)
        variants[fmt] = {"frame_period_p50_us": round(vp["p50_us"], 3), "p99_us": round(vp["p99_us"], 3),
                         "rms_jitter_us": round(vp["rms_jitter_us"], 3),
                         "frame_span_p50_us": round(vs["p50_us"], 3),
                         "matrix_MB": round(n_act * 2 * sc.n_valid * FMT_BYTES[fmt] / 1e6, 2),
                         "bytes_per_frame": vb,
                         "achieved_GBps": round(vb * args.launch_frames / (v["launch_ms"] * 1e6), 1)
                         if v["launches"] and args.variant_steps % args.launch_frames == 0 else None}
        rtc.rtc_destroy(vctx)
        log(f"{fmt}: frame period p50 {vp['p50_us']:.2f} us, p99 {vp['p99_us']:.2f} us")

    traffic = None
    if os.path.exists(PROFILE_TRAFFIC):
        try:
            prof = json.load(open(PROFILE_TRAFFIC))
            if (prof.get("kernel_source_sha256_16") == kernel_source_hash()
                    and prof.get("frames_per_launch") == args.launch_frames):
                traffic = prof.get("hbm_bytes_per_launch")
            elif prof.get("kernel_source_sha256_16") == kernel_source_hash():
                log(f"traffic counters were taken at {prof.get('frames_per_launch')} frames per launch; "
                    f"not reported for {args.launch_frames}")
        except Exception:
            traffic = None

    fb = frame_bytes(sc, "f32")
    full = args.steps % args.launch_frames == 0
    achieved = fb * args.launch_frames / (head["launch_ms"] * 1e6) if full else fb / (
        head["wall"] * 1e6 / args.steps) / 1e3
    result = {
        "metric": METRIC,
        "value": round(st_period["p50_us"], 3),
        "unit": "us",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["wall"] * 1e3 / args.steps, 6),
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
        "frame_period_us": st_period,
        "frame_span_us": st_span,
        "frame_period_us_skip100": frame_stats(head["period"], skip=100) if len(head["period"]) > 200 else None,
        "frame_period_us_within_launches": frame_stats(head["period_inside"]),
        "per_launch_mode": per_launch,
        "kernels_us": {"reconstruct_integrate": round(mvm_us, 3), "calibrate_centroid": round(cal_us, 3),
                       "frames_kernel_per_launch_ms": round(head["launch_ms"], 4)},
        "per_launch_gemv_GBps": round(mvm_bytes / mvm_us / 1e3, 1),
        "read_probe_GBps": probes,
        "precision_variants": variants,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                     "kernel": "frames_kernel (persistent: calibrate, CoG, R s, integrate)",
                     "bytes_per_frame": fb, "frames_per_launch": args.launch_frames,
                     "note": "algorithmic bytes; the kernel keeps part of the matrix in LDS and registers "
                             "across frames, so HBM traffic per frame is below the algorithmic bytes"},
    }
    if not args.no_cpu:
        log(f"timing the FP64 oracle for ~{args.cpu_seconds:.0f}s on the host")
        result["cpu_baseline"] = cpu_baseline(sc, ring, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
