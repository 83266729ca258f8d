"""Benchmark of the AO real-time-control frame on one MI355X.

One step = one ELT-scale SCAO frame through the whole hot path (calibration,
centre of gravity, control-matrix x slopes, integrator).  Frames run back to
back from a device-resident ring of pre-generated raw frames, as the paper's
no-camera measurements do; the per-frame device time stamps give the frame
time series (start of frame k to start of frame k+1) whose p50 is ``value``,
plus p99, RMS and peak-to-peak jitter.  The dominant kernel (the matrix-vector
reconstruction) is also timed alone with HIP events for the roofline figure,
and the FP64 oracle is timed on the host cores as a CPU baseline.

    python bench.py [--steps 10000] [--warmup 500] [--ring 128] [--k-split 1]
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
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "mvm_elt_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1805_07254_amd", "csrc", "rtc_kernels.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10000)
    p.add_argument("--warmup", type=int, default=500)
    p.add_argument("--ring", type=int, default=128, help="distinct raw frames kept on the device")
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


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
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

    ctx = rtc.rtc_init(sc.mask, cfg.n_pix, sc.n_act, gain=cfg.gain, leak=cfg.leak)
    rtc.rtc_load_calib(ctx, sc.dark, sc.flat, cfg.threshold)
    rtc.rtc_load_cmat(ctx, R)
    tuning = dict(kernel=args.mvm_kernel, k_split=args.k_split, rows_per_wave=args.rows_per_wave,
                  unroll=args.unroll, blocks=args.blocks, waves=args.waves)
    rtc.rtc_set_mvm_tuning(ctx, **tuning)
    khz = rtc.rtc_wall_clock_khz(ctx)
    dev_ring = torch.from_numpy(ring.reshape(args.ring, -1).view(np.int16)).to("cuda:0").view(torch.uint16)
    npx = cfg.frame_side * cfg.frame_side
    n_act = sc.n_act
    cmd = torch.empty(args.ring * n_act, dtype=torch.float32, device="cuda:0")
    ts = torch.zeros(2 * max(args.steps, 1), dtype=torch.int64, device="cuda:0")
    stream = torch.cuda.current_stream()

    def run(n, ts_buf=None):
        done = 0
        while done < n:
            m = min(args.ring, n - done)
            rtc.rtc_frame_batch(ctx, m, dev_ring, cmd, ts=None if ts_buf is None else ts_buf[2 * done:],
                                stream=stream)
            done += m

    run(args.warmup)
    torch.cuda.synchronize()
    log(f"warm-up {args.warmup} frames done; timing {args.steps} frames")
    t0 = time.perf_counter()
    run(args.steps, ts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stamps = ts.cpu().numpy().reshape(-1, 2)[:args.steps]
    start_us = ticks_to_us(stamps[:, 0] - stamps[0, 0], khz)
    end_us = ticks_to_us(stamps[:, 1] - stamps[0, 0], khz)
    period = np.diff(start_us)
    compute = end_us - start_us
    st_period = frame_stats(period)
    st_compute = frame_stats(compute)
    log(f"frame period p50 {st_period['p50_us']:.2f} us, compute p50 {st_compute['p50_us']:.2f} us, "
        f"wall {wall * 1e6 / args.steps:.2f} us/frame")

    # --- dominant kernel alone: reconstruction + integrator, HIP events on the launch stream
    slopes = torch.empty(2 * sc.n_valid, dtype=torch.float32, device="cuda:0")
    rtc.rtc_calibrate_centroid(ctx, dev_ring[0], slopes, stream=stream)
    out_cmd = torch.empty(n_act, dtype=torch.float32, device="cuda:0")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # raw addresses keep the host-side cost per launch far below a kernel's duration
    s_ptr, c_ptr, st_ptr = slopes.data_ptr(), out_cmd.data_ptr(), stream.cuda_stream
    frame_ptrs = [dev_ring[i].data_ptr() for i in range(args.ring)]
    for _ in range(50):
        rtc.rtc_reconstruct_integrate(ctx, s_ptr, c_ptr, stream=st_ptr)
    ev0.record(stream)
    for _ in range(args.kernel_reps):
        rtc.rtc_reconstruct_integrate(ctx, s_ptr, c_ptr, stream=st_ptr)
    ev1.record(stream)
    ev1.synchronize()
    mvm_us = ev0.elapsed_time(ev1) * 1e3 / args.kernel_reps
    ev0.record(stream)
    for i in range(args.kernel_reps):
        rtc.rtc_calibrate_centroid(ctx, frame_ptrs[i % args.ring], s_ptr, stream=st_ptr)
    ev1.record(stream)
    ev1.synchronize()
    cal_us = ev0.elapsed_time(ev1) * 1e3 / args.kernel_reps
    ldr = (2 * sc.n_valid + 3) // 4 * 4
    mvm_bytes = n_act * ldr * 4 + ldr * 4 + 3 * n_act * 4        # R, s, state r/w, cmd w
    cal_bytes = sc.n_valid * cfg.n_pix ** 2 * (2 + 8) + sc.n_valid * (2 * 4 + 4) + sc.n_valid * 2 * 4
    log(f"reconstruct+integrate {mvm_us:.2f} us/launch ({mvm_bytes / mvm_us / 1e3:.0f} GB/s), "
        f"calibrate+centroid {cal_us:.2f} us/launch")

    # --- read-bandwidth probes at the matrix's working-set size and at 2 GB
    probes = {}
    out1 = torch.zeros(1, dtype=torch.float32, device="cuda:0")
    for label, nbytes in (("140MB", mvm_bytes // 16 * 16), ("2GB", 2 << 30)):
        buf = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
        for _ in range(5):
            rtc.rtc_probe_read(ctx, buf, nbytes, out1, stream=stream)
        reps = 200 if nbytes < (1 << 30) else 20
        ev0.record(stream)
        for _ in range(reps):
            rtc.rtc_probe_read(ctx, buf, nbytes, out1, stream=stream)
        ev1.record(stream)
        ev1.synchronize()
        us = ev0.elapsed_time(ev1) * 1e3 / reps
        probes[label] = round(nbytes / us / 1e3, 1)
        del buf
    # plain copy of known size: the reference for scaling HBM byte counters
    copy_bytes = 256 << 20
    src = torch.empty(copy_bytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    rtc.rtc_probe_copy(ctx, src, dst, copy_bytes, stream=stream)
    ev0.record(stream)
    for _ in range(10):
        rtc.rtc_probe_copy(ctx, src, dst, copy_bytes, stream=stream)
    ev1.record(stream)
    ev1.synchronize()
    probes["copy_256MiB"] = round(2 * copy_bytes / (ev0.elapsed_time(ev1) * 1e3 / 10) / 1e3, 1)
    del src, dst
    log(f"read/copy probes GB/s: {probes}")

    # --- reduced-precision control matrices: same frames, same launch shape
    variants = {}
    for fmt in [v for v in args.variants.split(",") if v]:
        vctx = rtc.rtc_init(sc.mask, cfg.n_pix, sc.n_act, cm_dtype=fmt, gain=cfg.gain, leak=cfg.leak)
        rtc.rtc_load_calib(vctx, sc.dark, sc.flat, cfg.threshold)
        rtc.rtc_load_cmat(vctx, R)
        rtc.rtc_set_mvm_tuning(vctx, **{k: v for k, v in tuning.items() if k != "kernel"})
        nf = args.variant_steps
        vts = torch.zeros(2 * nf, dtype=torch.int64, device="cuda:0")
        done = 0
        while done < 200:
            m = min(args.ring, 200 - done)
            rtc.rtc_frame_batch(vctx, m, dev_ring, cmd, stream=stream)
            done += m
        done = 0
        while done < nf:
            m = min(args.ring, nf - done)
            rtc.rtc_frame_batch(vctx, m, dev_ring, cmd, ts=vts[2 * done:], stream=stream)
            done += m
        torch.cuda.synchronize()
        vst = vts.cpu().numpy().reshape(-1, 2)
        vper = frame_stats(np.diff(ticks_to_us(vst[:, 0] - vst[0, 0], khz)))
        for _ in range(50):
            rtc.rtc_reconstruct_integrate(vctx, s_ptr, c_ptr, stream=st_ptr)
        ev0.record(stream)
        for _ in range(args.kernel_reps):
            rtc.rtc_reconstruct_integrate(vctx, s_ptr, c_ptr, stream=st_ptr)
        ev1.record(stream)
        ev1.synchronize()
        v_us = ev0.elapsed_time(ev1) * 1e3 / args.kernel_reps
        esz = {"f16": 2, "bf16": 2, "fp8e4m3": 1}[fmt]
        epc = 16 // esz
        ldq = (2 * sc.n_valid + epc - 1) // epc * epc
        v_bytes = n_act * ldq * esz + n_act * 4 + ldq * 4 + 3 * n_act * 4   # codes, scales, slopes, state, cmd
        variants[fmt] = {"frame_period_p50_us": round(vper["p50_us"], 3), "p99_us": round(vper["p99_us"], 3),
                         "rms_jitter_us": round(vper["rms_jitter_us"], 3),
                         "reconstruct_integrate_us": round(v_us, 3),
                         "matrix_MB": round(n_act * ldq * esz / 1e6, 2),
                         "achieved_GBps": round(v_bytes / v_us / 1e3, 1),
                         "frac_of_hbm_peak": round(v_bytes / v_us / 1e3 / HBM_PEAK_GBPS, 4)}
        rtc.rtc_destroy(vctx)
        log(f"{fmt}: frame p50 {vper['p50_us']:.2f} us, reconstruction {v_us:.2f} us "
            f"({variants[fmt]['achieved_GBps']:.0f} GB/s)")

    traffic = None
    if os.path.exists(PROFILE_TRAFFIC):
        try:
            prof = json.load(open(PROFILE_TRAFFIC))
            if prof.get("kernel_source_sha256_16") == kernel_source_hash():
                traffic = prof.get("hbm_bytes_per_launch")
        except Exception:
            traffic = None

    achieved = mvm_bytes / mvm_us / 1e3
    result = {
        "metric": METRIC,
        "value": round(st_period["p50_us"], 3),
        "unit": "us",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 6),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{cfg.name}: {cfg.n_sub}x{cfg.n_sub} SH, {cfg.n_pix}x{cfg.n_pix} px, "
                        f"obscuration {cfg.obscuration}, {sc.n_valid} subapertures, {2 * sc.n_valid} slopes, "
                        f"{sc.n_act} actuators, FP32 control matrix {R.nbytes / 1e6:.1f} MB",
            "frames_ring": args.ring,
            "mvm_tuning": tuning,
            "frame_data": "open-loop frozen-flow von Karman frames (r0 0.15 m, L0 25 m, 10 m/s)",
        },
        "frame_period_us": st_period,
        "frame_compute_us": st_compute,
        "frame_period_us_skip100": frame_stats(period, skip=100) if len(period) > 200 else None,
        "gemv_GBps": round(achieved, 1),
        "kernels_us": {"reconstruct_integrate": round(mvm_us, 3), "calibrate_centroid": round(cal_us, 3)},
        "read_probe_GBps": probes,
        "precision_variants": variants,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                     "kernel": "mvm_kernel (reconstruct + integrate)",
                     "bytes_per_launch": int(mvm_bytes)},
    }
    if not args.no_cpu:
        log(f"timing the FP64 oracle for ~{args.cpu_seconds:.0f}s on the host")
        result["cpu_baseline"] = cpu_baseline(sc, ring, args.cpu_seconds)
    rtc.rtc_destroy(ctx)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
