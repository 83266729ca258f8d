// C-ABI host side of pixel-stream processing (declared in include/rtc.h):
// subaperture allocation, column-major copy of the control matrix, and the
// launch of the camera emulator + workers (Section 2.3.6, Figure 6).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "rtc_ctx.h"

using namespace rtcx;

namespace {

namespace pl = rtck::pipe_layout;

constexpr double kLeadUs = 200.0;        // camera start to frame 0: workers copy their LDS columns meanwhile
constexpr double kWaitSlackUs = 50000.0;

// Linearly decreasing counts (see rtc_pipe_allocation).
void linear_allocation(int32_t n, int32_t P, double ratio, int32_t *counts) {
  std::vector<double> w(P), frac(P);
  double sw = 0.0;
  for (int32_t b = 0; b < P; ++b) {
    w[b] = P == 1 ? 1.0 : ratio + (1.0 - ratio) * (double)b / (double)(P - 1);
    sw += w[b];
  }
  int64_t assigned = 0;
  for (int32_t b = 0; b < P; ++b) {
    const double x = (double)n * w[b] / sw;
    const double fl = std::floor(x);
    counts[b] = (int32_t)fl;
    frac[b] = x - fl;
    assigned += counts[b];
  }
  std::vector<int32_t> order(P);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return frac[a] > frac[b]; });
  for (int64_t i = 0; i < (int64_t)n - assigned; ++i) counts[order[i % P]] += 1;
}

}  // namespace

extern "C" {

rtc_status rtc_pipe_allocation(int32_t n_subaps, int32_t n_workers, double ratio, int32_t *counts) {
  if (!counts) return fail(nullptr, RTC_E_ARG, "rtc_pipe_allocation: NULL counts");
  if (n_subaps < 0 || n_workers < 1) return fail(nullptr, RTC_E_ARG, "rtc_pipe_allocation: n_subaps < 0 or n_workers < 1");
  if (!(ratio >= 1.0 && ratio <= 1000.0)) return fail(nullptr, RTC_E_ARG, "rtc_pipe_allocation: ratio outside [1, 1000]");
  linear_allocation(n_subaps, n_workers, ratio, counts);
  return RTC_OK;
}

rtc_status rtc_pipe_setup(rtc_ctx *c, const rtc_pipe_config *cfg) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_pipe_setup: NULL context");
  if (!cfg) return fail(c, RTC_E_ARG, "rtc_pipe_setup: NULL config");
  if (!c->cmat_loaded) return fail(c, RTC_E_STATE, "rtc_pipe_setup: load the control matrix first");
  if (cfg->full_frame != 0 && cfg->full_frame != 1) return fail(c, RTC_E_ARG, "rtc_pipe_setup: full_frame must be 0 or 1");
  if (!(cfg->alloc_ratio >= 1.0 && cfg->alloc_ratio <= 1000.0))
    return fail(c, RTC_E_ARG, "rtc_pipe_setup: alloc_ratio outside [1, 1000]");
  if (!(cfg->frame_period_us > 0.0 && cfg->frame_period_us <= 1e6))
    return fail(c, RTC_E_ARG, "rtc_pipe_setup: frame_period_us outside (0, 1e6]");
  if (!(cfg->readout_us > 0.0 && cfg->readout_us <= cfg->frame_period_us))
    return fail(c, RTC_E_ARG, "rtc_pipe_setup: readout_us outside (0, frame_period_us]");
  if (cfg->rows_per_packet < 1) return fail(c, RTC_E_ARG, "rtc_pipe_setup: rows_per_packet < 1");
  if (cfg->wait_limit_us < 0) return fail(c, RTC_E_ARG, "rtc_pipe_setup: wait_limit_us < 0");
  if (cfg->reserved != 0) return fail(c, RTC_E_ARG, "rtc_pipe_setup: reserved must be 0");
  if (cfg->n_workers < 0) return fail(c, RTC_E_ARG, "rtc_pipe_setup: n_workers < 0");
  const int32_t P = cfg->n_workers > 0 ? cfg->n_workers : c->n_cu - 1;
  if (P < 1 || P + 1 > c->n_cu || P > pl::kMaxWorkers)
    return fail(c, RTC_E_ARG, "rtc_pipe_setup: n_workers must leave one compute unit for the camera");
  if (c->wfs.size() != 1) return fail(c, RTC_E_UNSUPPORTED, "rtc_pipe_setup: one wavefront sensor only");
  if (c->n_act > 8192) return fail(c, RTC_E_UNSUPPORTED, "rtc_pipe_setup: more than 8192 actuators");
  if ((c->n_act + P - 1) / P > 64) return fail(c, RTC_E_UNSUPPORTED, "rtc_pipe_setup: more than 64 actuator rows per worker");
  if (c->frame_elems % 2 != 0) return fail(c, RTC_E_UNSUPPORTED, "rtc_pipe_setup: odd frame size");

  const WfsInfo &wi = c->wfs[0];
  if (cfg->tail_rows < 0 || cfg->tail_rows > wi.n_sub_y)
    return fail(c, RTC_E_ARG, "rtc_pipe_setup: tail_rows outside [0, n_sub_y]");
  const int32_t n = c->n_valid;
  // tail: the subapertures of the last tail_rows rows (a suffix of the row-major order)
  const int32_t tail_top = wi.H - cfg->tail_rows * wi.n_pix;
  int32_t n_main = n;
  while (n_main > 0 && c->tiles_h[n_main - 1].off / c->tiles_h[n_main - 1].pitch >= tail_top) --n_main;
  const int32_t n_tail = n - n_main;
  if (n_tail > rtck::kPipeMaxTail) return fail(c, RTC_E_UNSUPPORTED, "rtc_pipe_setup: more than 64 tail subapertures");
  // owners: the first half of the workers (at least enough for 64 rows each)
  const int32_t n_own = std::min(P, std::max((c->n_act + 63) / 64, (P + 1) / 2));
  const int32_t own_max = (c->n_act + n_own - 1) / n_own;
  std::vector<int32_t> counts(P), first(P + 1, 0), need(n);
  linear_allocation(n_main, P, cfg->alloc_ratio, counts.data());
  int32_t max_nb = 1;
  for (int32_t b = 0; b < P; ++b) {
    first[b + 1] = first[b] + counts[b];
    max_nb = std::max(max_nb, counts[b]);
  }
  for (int32_t k = 0; k < n; ++k) {
    const rtck::TileDesc &t = c->tiles_h[k];
    need[k] = cfg->full_frame ? wi.H : t.off / t.pitch + t.n;
  }

  DeviceScope ds(c->device);
  if (ds.status != hipSuccess) return hip_fail(c, ds.status, "rtc_pipe_setup: hipSetDevice");
  int lds_max = 0;
  hipError_t e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device);
  if (e != hipSuccess) return hip_fail(c, e, "rtc_pipe_setup: device attributes");
  const int code_bytes = rtck::format_code_bytes(c->fmt);
  const int64_t ldp = (c->n_act + 63) / 64 * 64;
  const int64_t col_bytes = ldp * code_bytes;
  const size_t fixed = rtck::pipe_lds_fixed(max_nb, n_tail, own_max);
  const int64_t avail = (int64_t)lds_max - (int64_t)fixed - rtck::kPipeStaticLds;
  if (avail < 0) return fail(c, RTC_E_UNSUPPORTED, "rtc_pipe_setup: too many subapertures per worker for LDS");
  const int32_t lds_cols = (int32_t)std::min<int64_t>(2 * (int64_t)max_nb, avail / col_bytes);
  const size_t lds = (size_t)lds_cols * col_bytes + fixed;
  const int64_t ring_stride = (c->frame_elems + 127) / 128 * 128;

  void *d_packed = nullptr;
  float *d_ppart = nullptr;
  uint16_t *d_ring = nullptr;
  uint32_t *d_psync = nullptr;
  int32_t *d_first = nullptr, *d_need = nullptr;
  auto release = [&]() {
    dfree(d_packed);
    dfree(d_ppart);
    dfree(d_ring);
    dfree(d_psync);
    dfree(d_first);
    dfree(d_need);
  };
  if (e == hipSuccess) e = hipMalloc(&d_packed, (size_t)2 * n * col_bytes);
  if (e == hipSuccess) e = hipMalloc(&d_ppart, (size_t)2 * P * ldp * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&d_ring, (size_t)2 * ring_stride * sizeof(uint16_t));
  if (e == hipSuccess) e = hipMalloc(&d_psync, (size_t)pl::kWords * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&d_first, (size_t)(P + 1) * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc(&d_need, (size_t)n * sizeof(int32_t));
  if (e != hipSuccess) {
    release();
    return hip_fail(c, e, "rtc_pipe_setup: hipMalloc");
  }
  if ((e = hipDeviceSynchronize()) == hipSuccess &&
      (e = hipMemset(d_ppart, 0, (size_t)2 * P * ldp * sizeof(float))) == hipSuccess &&
      (e = hipMemset(d_ring, 0, (size_t)2 * ring_stride * sizeof(uint16_t))) == hipSuccess &&
      (e = hipMemset(d_psync, 0, (size_t)pl::kWords * sizeof(uint32_t))) == hipSuccess &&
      (e = hipMemcpy(d_first, first.data(), (size_t)(P + 1) * sizeof(int32_t), hipMemcpyHostToDevice)) == hipSuccess &&
      (e = hipMemcpy(d_need, need.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice)) == hipSuccess)
    e = rtck::launch_pack_columns(c->d_R, c->ldq * code_bytes, c->fmt, c->d_tiles, n, c->n_act, d_packed, ldp,
                                  nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    release();
    return hip_fail(c, e, "rtc_pipe_setup: upload");
  }
  dfree(c->d_packed);
  dfree(c->d_ppart);
  dfree(c->d_ring);
  dfree(c->d_psync);
  dfree(c->d_first);
  dfree(c->d_need);
  c->d_packed = d_packed;
  c->d_ppart = d_ppart;
  c->d_ring = d_ring;
  c->d_psync = d_psync;
  c->d_first = d_first;
  c->d_need = d_need;
  c->pipe_cfg = *cfg;
  c->pipe_workers = P;
  c->pipe_lds_cols = lds_cols;
  c->pipe_max_nb = max_nb;
  c->pipe_n_tail = n_tail;
  c->pipe_own_max = own_max;
  c->pipe_n_own = n_own;
  c->pipe_H = wi.H;
  c->pipe_W = wi.W;
  c->pipe_ldp = ldp;
  c->pipe_ring_stride = ring_stride;
  c->pipe_lds = lds;
  c->pipe_gen = c->cmat_gen;
  return RTC_OK;
}

rtc_status rtc_pipe_info(const rtc_ctx *c, int32_t *n_workers, int32_t *lds_cols, int32_t *image_rows,
                         int32_t *max_subaps, int32_t *n_tail, int32_t *n_owners) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_pipe_info: NULL context");
  if (c->pipe_gen == 0) return fail(const_cast<rtc_ctx *>(c), RTC_E_STATE, "rtc_pipe_info: call rtc_pipe_setup first");
  if (n_workers) *n_workers = c->pipe_workers;
  if (lds_cols) *lds_cols = c->pipe_lds_cols;
  if (image_rows) *image_rows = c->pipe_H;
  if (max_subaps) *max_subaps = c->pipe_max_nb;
  if (n_tail) *n_tail = c->pipe_n_tail;
  if (n_owners) *n_owners = c->pipe_n_own;
  return RTC_OK;
}

rtc_status rtc_pipe_run(rtc_ctx *c, int32_t n_frames, const uint16_t *d_frames, int64_t frame_stride,
                        float *d_cmd, float *d_slopes, float *d_recon, int32_t *d_counts, uint64_t *d_cam_ts,
                        uint64_t *d_worker_ts, void *hip_stream) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_pipe_run: NULL context");
  if (!c->calib_loaded) return fail(c, RTC_E_STATE, "rtc_pipe_run: load the calibration first");
  if (c->pipe_gen == 0 || c->pipe_gen != c->cmat_gen)
    return fail(c, RTC_E_STATE, "rtc_pipe_run: call rtc_pipe_setup after loading the control matrix");
  if (c->state_invalid) return fail(c, RTC_E_STATE, "rtc_pipe_run: " STATE_INVALID_MSG);
  if (!c->dark_fast)
    return fail(c, RTC_E_UNSUPPORTED, "rtc_pipe_run: pixel-stream processing needs every dark to be 0 or of "
                                      "magnitude in [2^-13, 2^24)");
  if (n_frames < 0) return fail(c, RTC_E_ARG, "rtc_pipe_run: n_frames < 0");
  if (n_frames == 0) return RTC_OK;
  if (!d_frames || !d_cmd) return fail(c, RTC_E_ARG, "rtc_pipe_run: NULL frames or cmd");
  if (frame_stride < c->frame_elems || frame_stride % 2 != 0)
    return fail(c, RTC_E_ARG, "rtc_pipe_run: frame_stride must be even and >= the frame size");
  if ((reinterpret_cast<uintptr_t>(d_frames) & 3) != 0)
    return fail(c, RTC_E_ARG, "rtc_pipe_run: frames must be 4-byte aligned");
  const int32_t P = c->pipe_workers;
  if ((int64_t)n_frames * c->pipe_H >= (int64_t)1 << 31 || (int64_t)P * (n_frames + 1) >= (int64_t)1 << 31)
    return fail(c, RTC_E_ARG, "rtc_pipe_run: too many frames for one launch");
  DeviceScope ds(c->device);
  if (ds.status != hipSuccess) return hip_fail(c, ds.status, "rtc_pipe_run: hipSetDevice");
  const rtc_pipe_config &cfg = c->pipe_cfg;
  const double tpu = (double)c->wall_khz / 1000.0;   // ticks per microsecond
  rtck::PipeArgs p{};
  p.tiles = c->d_tiles;
  p.calib = c->d_calib;
  p.ref = c->d_ref;
  p.n_valid = c->n_valid;
  p.max_n = c->max_n;
  p.mode = c->cfg.thr_mode;
  p.dark_fast = c->dark_fast;
  p.fmt = c->fmt;
  p.src = d_frames;
  p.src_stride = frame_stride;
  p.ring = c->d_ring;
  p.ring_stride = c->pipe_ring_stride;
  p.frame_elems = c->frame_elems;
  p.H = c->pipe_H;
  p.W = c->pipe_W;
  p.rows_per_packet = cfg.rows_per_packet;
  p.n_frames = n_frames;
  p.t_frame = cfg.frame_period_us * tpu;
  p.t_row = cfg.readout_us * tpu / (double)c->pipe_H;
  p.lead = (int64_t)(kLeadUs * tpu);
  p.wait_ticks = cfg.wait_limit_us > 0 ? (int64_t)(cfg.wait_limit_us * tpu)
                                       : (int64_t)((2.0 * cfg.frame_period_us + kLeadUs + kWaitSlackUs) * tpu);
  p.first = c->d_first;
  p.need = c->d_need;
  p.packed = c->d_packed;
  p.ldp = c->pipe_ldp;
  p.lds_cols = c->pipe_lds_cols;
  p.max_nb = c->pipe_max_nb;
  p.n_tail = c->pipe_n_tail;
  p.own_max = c->pipe_own_max;
  p.n_own = c->pipe_n_own;
  p.n_act = c->n_act;
  p.scales = c->d_scales;
  p.state = c->d_state;
  p.cmd = d_cmd;
  p.recon = d_recon;
  p.gain = c->cfg.gain;
  p.leak = c->cfg.leak;
  p.cmd_min = c->cfg.cmd_min;
  p.cmd_max = c->cfg.cmd_max;
  p.part = c->d_ppart;
  p.s_user = d_slopes;
  p.counts = d_counts;
  p.sync = c->d_psync;
  p.abort_flag = c->d_sync + rtck::sync_layout::kAbort;
  p.sticky = c->d_sync + rtck::sync_layout::kSticky;
  p.cam_ts = d_cam_ts;
  p.wk_ts = d_worker_ts;
  const hipError_t e = rtck::launch_pipe(p, P + 1, c->pipe_lds, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? RTC_OK : hip_fail(c, e, "rtc_pipe_run: launch");
}

}  // extern "C"
