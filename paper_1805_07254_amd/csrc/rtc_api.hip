// C-ABI host side of the SH-WFS real-time-control library (declared in include/rtc.h).
//
// Validation happens on the host before any device state changes, so every
// error leaves the context as it was.  Device buffers:
//   tiles    [n_valid]            TileDesc of each active subaperture (offsets, slope positions, threshold)
//   calib    per tile [n][n]      float2 (dark, flat), active tiles only
//   ref      [s_len]              float32 reference slopes, s_len = round_up(2 n_valid, 16), zero-padded
//   R        [n_act][ldq]         codes of the storage format, ldq = round_up(2 n_valid, elements per
//                                 16 bytes), zero-padded; float32 storage has ldq = round_up(2 n_valid, 4)
//   scales   [n_act]              float32 per-row scales (reduced formats only)
//   s        [s_len]              float32 slope vector of the current frame, zero-padded
//   state    [n_act]              float32 integrator state
//   part     [64][n_act]          float32 split-K partial actuator vectors
//   sync     [4]                  uint32 completion counter
#include <hip/hip_runtime.h>

#include <time.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/rtc.h"
#include "rtc_kernels.h"

#include "rtc_ctx.h"

using namespace rtcx;

namespace {

bool dark_in_domain(float d) {
  // raw - dark is exact in float64 for every raw in [0, 65535] when this holds;
  // other darks take the kernels' exact slow path.
  const float a = std::fabs(d);
  return d == 0.0f || (a >= 0x1p-13f && a < 0x1p24f);
}

// Slope exchange buffer of persistent batches: whole groups of 64 chunks of
// the largest chunk (16 elements), so every format's layout fits.
int64_t xchg_len_of(int64_t n_slopes) { return (n_slopes + 1023) / 1024 * 1024; }

constexpr int kSyncWords = rtck::sync_layout::kWords;

int64_t round_up4(int64_t x) { return (x + 3) & ~int64_t(3); }
int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Storage formats: exponent bits, fraction bits, bias, E (row scales map the row
// maximum into (2^(E-1), 2^E]), bytes per element.
struct FmtDesc {
  int ebits, fbits, bias, E, bytes;
};
const FmtDesc kFmt[4] = {{8, 23, 127, 0, 4}, {5, 10, 15, 15, 2}, {8, 7, 127, 0, 2}, {4, 3, 7, 8, 1}};

// Round-to-nearest-even of |y| (finite, within the format's range) onto the
// format's grid, then the bit pattern of the result.
uint32_t encode_value(double y, const FmtDesc &f) {
  const uint32_t sign = std::signbit(y) ? 1u : 0u;
  const int sign_shift = f.ebits + f.fbits;
  const double a = std::fabs(y);
  if (a == 0.0) return sign << sign_shift;
  int ex = 0;
  (void)std::frexp(a, &ex);                         // a in [2^(ex-1), 2^ex)
  const int e_unb = std::max(ex - 1, 1 - f.bias);
  const double q = std::ldexp(1.0, e_unb - f.fbits);
  const double v = std::nearbyint(a / q) * q;      // a / q exact; nearbyint ties to even
  if (v == 0.0) return sign << sign_shift;
  int ev = 0;
  (void)std::frexp(v, &ev);
  uint32_t e_field, frac;
  if (v >= std::ldexp(1.0, 1 - f.bias)) {
    e_field = (uint32_t)(ev - 1 + f.bias);
    frac = (uint32_t)(std::ldexp(v, -(ev - 1) + f.fbits) - std::ldexp(1.0, f.fbits));
  } else {
    e_field = 0;
    frac = (uint32_t)std::ldexp(v, f.bias - 1 + f.fbits);
  }
  return (sign << sign_shift) | (e_field << f.fbits) | frac;
}

// Smallest e with max|row| / 2^e <= 2^E, clamped to [-126, 127]; 0 for a zero row.
int row_scale_exponent(const float *row, int32_t n, const FmtDesc &f) {
  double m = 0.0;
  for (int32_t j = 0; j < n; ++j) m = std::max(m, (double)std::fabs(row[j]));
  if (m == 0.0) return 0;
  int p = 0;
  const double mant = std::frexp(m, &p);
  const int ceil_log2 = (mant == 0.5) ? p - 1 : p;
  return std::min(127, std::max(-126, ceil_log2 - f.E));
}

// Encodes rows [0, n_rows) of R (row pitch ld) into codes with row pitch
// ldc elements (columns n_cols..ldc-1 are zero codes) and per-row scales.
void encode_rows(int fmt, const float *R, int32_t n_rows, int32_t n_cols, int64_t ld, void *codes, int64_t ldc,
                 float *scales) {
  const FmtDesc &f = kFmt[fmt];
  for (int32_t r = 0; r < n_rows; ++r) {
    const float *row = R + (int64_t)r * ld;
    const int e = row_scale_exponent(row, n_cols, f);
    scales[r] = std::ldexp(1.0f, e);
    for (int64_t j = 0; j < ldc; ++j) {
      const uint32_t code = j < n_cols ? encode_value(std::ldexp((double)row[j], -e), f) : 0u;
      if (f.bytes == 2)
        static_cast<uint16_t *>(codes)[(int64_t)r * ldc + j] = (uint16_t)code;
      else
        static_cast<uint8_t *>(codes)[(int64_t)r * ldc + j] = (uint8_t)code;
    }
  }
}

// Scratch of rtc_frame_batch_noalloc: a code-object array, so every device
// the library runs on holds its own copy from module load to process exit and
// no call allocates it.  Host code never passes `scratch` itself (its host
// name is only a stand-in): the device address is taken once per device with
// hipGetSymbolAddress when a context is created there.  Every such call on a
// device shares that device's copy.  Layout in uint32 words, every region
// starting on a 256-byte boundary:
//   [0, 64)               completion counter (word 0) and abort flag (word 1)
//   sbuf  [2][xchg_len]   slope vectors of consecutive frames (persistent batches)
//   s     [s_len]         slope vector of the current frame (per-launch frames)
//   part  [k_split][n_act] split-K partial actuator vectors (per-launch frames)
//   bar   [kWords - kBarBase] barrier counters, mailboxes and end stamps
// The first three regions are zeroed by a kernel at the start of every call;
// the barrier words are zeroed before every persistent launch.
constexpr int64_t kScratchWords = int64_t(1) << 20;   // 4 MiB
static __device__ __align__(256) uint32_t scratch[kScratchWords];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
uint32_t *g_scratch_ptr[kScratchDevices] = {};

// Device address of this device's scratch array, resolved on first use; `dev`
// must be current.  Devices beyond the table get nullptr (no such entry point).
hipError_t scratch_address(int dev, uint32_t **out) {
  *out = nullptr;
  if (dev < 0 || dev >= kScratchDevices) return hipSuccess;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<uint32_t *>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

struct ScratchLayout {
  int64_t sbuf, s, part, bar, zero_words, words;
};

ScratchLayout scratch_layout(const rtc_ctx *c) {
  ScratchLayout L{};
  L.sbuf = 64;
  L.s = L.sbuf + 2 * xchg_len_of(c->n_slopes);
  L.part = L.s + round_up(c->s_len, 64);
  L.bar = L.part + round_up((int64_t)c->tuning.k_split * c->n_act, 64);
  L.zero_words = L.part;
  L.words = L.bar + (kSyncWords - rtck::sync_layout::kBarBase);
  return L;
}

// Per-frame scratch of the per-launch path.
struct FrameScratch {
  float *s;
  float *part;
  uint32_t *sync;
};

}  // namespace

extern "C" {

static bool horiz_shape(const rtc_ctx *c, int32_t *nch, int32_t *nrt, int32_t *nq, std::string *why);
static rtc_status horiz_prepare(rtc_ctx *c, const char *who);

uint32_t rtc_abi_version(void) { return RTC_ABI_VERSION; }

const char *rtc_error_string(const rtc_ctx *c) {
  return c ? c->err.c_str() : g_init_err.c_str();
}

int32_t rtc_n_valid(const rtc_ctx *c) { return c ? c->n_valid : -1; }
int32_t rtc_n_act(const rtc_ctx *c) { return c ? c->n_act : -1; }

// Common initialisation of one or more sensors; cfg holds the non-sensor fields.
static rtc_status init_impl(const rtc_config *cfg, const rtc_wfs *wfs, int32_t n_wfs, const char *who,
                            rtc_ctx **out) {
  auto err = [&](rtc_status st, const char *msg) { return fail(nullptr, st, std::string(who) + ": " + msg); };
  if (cfg->abi_version != RTC_ABI_VERSION) return err(RTC_E_ARG, "abi_version does not match RTC_ABI_VERSION");
  if (n_wfs < 1 || n_wfs > 64 || !wfs) return err(RTC_E_ARG, "n_wfs must be in 1..64 with a sensor array");
  std::vector<WfsInfo> info((size_t)n_wfs);
  std::vector<rtck::TileDesc> tiles;
  int64_t frame_elems = 0, calib_len = 0;
  int32_t max_n = 0;
  bool pairs = true;
  for (int32_t w = 0; w < n_wfs; ++w) {
    const rtc_wfs &d = wfs[w];
    if (d.n_sub_x < 1 || d.n_sub_x > 4096 || d.n_sub_y < 1 || d.n_sub_y > 4096)
      return err(RTC_E_ARG, "n_sub_x/n_sub_y must be in 1..4096");
    if (d.n_pix < 1 || d.n_pix > 32) return err(RTC_E_ARG, "n_pix must be in 1..32");
    if (!d.subap_mask) return err(RTC_E_ARG, "subap_mask is NULL");
    WfsInfo &wi = info[w];
    wi.n_sub_x = d.n_sub_x;
    wi.n_sub_y = d.n_sub_y;
    wi.n_pix = d.n_pix;
    wi.H = d.n_sub_y * d.n_pix;
    wi.W = d.n_sub_x * d.n_pix;
    wi.frame_off = frame_elems;
    wi.tile_base = (int32_t)tiles.size();
    frame_elems += (int64_t)wi.H * wi.W;
    if (frame_elems >= (int64_t(1) << 31)) return err(RTC_E_ARG, "the frame set has 2^31 or more pixels");
    max_n = std::max(max_n, d.n_pix);
    if ((d.n_pix & 1) || (wi.W & 1) || (wi.frame_off & 1)) pairs = false;
    // active subapertures row-major; slope positions are fixed once all sensors are known
    for (int32_t sy = 0; sy < d.n_sub_y; ++sy)
      for (int32_t sx = 0; sx < d.n_sub_x; ++sx)
        if (d.subap_mask[(int64_t)sy * d.n_sub_x + sx]) {
          rtck::TileDesc t{};
          t.off = (int32_t)(wi.frame_off + (int64_t)sy * d.n_pix * wi.W + (int64_t)sx * d.n_pix);
          t.calib_off = (int32_t)calib_len;
          t.pitch = wi.W;
          t.n = d.n_pix;
          t.thr = 0.0f;
          calib_len += (int64_t)d.n_pix * d.n_pix;
          tiles.push_back(t);
        }
    wi.n_tiles = (int32_t)tiles.size() - wi.tile_base;
    if (wi.n_tiles == 0) return err(RTC_E_ARG, "the mask has no active subaperture");
  }
  if (calib_len >= (int64_t(1) << 31)) return err(RTC_E_ARG, "calibration blocks too large");
  const int32_t n_valid = (int32_t)tiles.size();
  for (const WfsInfo &wi : info)                   // each sensor: its x block, then its y block
    for (int32_t k = 0; k < wi.n_tiles; ++k) {
      rtck::TileDesc &t = tiles[(size_t)wi.tile_base + k];
      t.sx = 2 * wi.tile_base + k;
      t.sy = 2 * wi.tile_base + wi.n_tiles + k;
    }
  if (cfg->n_act < 1 || cfg->n_act > (1 << 20)) return err(RTC_E_ARG, "n_act must be in 1..2^20");
  if (cfg->thr_mode != RTC_THR_NONE && cfg->thr_mode != RTC_THR_SUBTRACT && cfg->thr_mode != RTC_THR_ZERO)
    return err(RTC_E_ARG, "thr_mode must be RTC_THR_NONE, RTC_THR_SUBTRACT or RTC_THR_ZERO");
  if (cfg->cm_dtype < RTC_CM_F32 || cfg->cm_dtype > RTC_CM_FP8E4M3) return err(RTC_E_ARG, "unknown cm_dtype");
  if (!std::isfinite(cfg->gain) || !std::isfinite(cfg->leak))
    return err(RTC_E_NONFINITE, "gain and leak must be finite");
  if (std::isnan(cfg->cmd_min) || std::isnan(cfg->cmd_max)) return err(RTC_E_NONFINITE, "cmd_min/cmd_max must not be NaN");
  if (!(cfg->cmd_min <= cfg->cmd_max)) return err(RTC_E_ARG, "cmd_min > cmd_max");
  if (cfg->device < 0) return err(RTC_E_ARG, "device must be >= 0");
  if (cfg->cm_dtype != RTC_CM_F32) {
    // reduced formats run on the row-block kernels: slices of 8 wavefronts in panels
    const int epc = rtck::format_elems_per_chunk(cfg->cm_dtype);
    const int64_t chunks = round_up(2 * (int64_t)n_valid, epc) / epc;
    if (chunks > (int64_t)1 << 24) return err(RTC_E_UNSUPPORTED, "slope vector too long for a reduced-precision matrix");
  }

  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0)
    return fail(nullptr, RTC_E_DEVICE, std::string(who) + ": no HIP device available (" +
                                           (e != hipSuccess ? hipGetErrorName(e) : "count 0") + ")");
  if (cfg->device >= ndev) return err(RTC_E_DEVICE, "device ordinal out of range");

  rtc_ctx *c = new (std::nothrow) rtc_ctx();
  if (!c) return err(RTC_E_NOMEM, "host allocation failed");
  c->cfg = *cfg;
  c->cfg.subap_mask = nullptr;
  c->device = cfg->device;
  c->wfs = std::move(info);
  c->frame_elems = frame_elems;
  c->max_n = max_n;
  c->pairs = pairs ? 1 : 0;
  c->calib_len = calib_len;
  c->n_valid = n_valid;
  c->n_slopes = 2 * n_valid;
  c->ldr = round_up4(c->n_slopes);
  c->n_s4 = (int32_t)(c->ldr / 4);
  c->s_len = round_up(c->n_slopes, 16);
  c->fmt = cfg->cm_dtype;
  {
    const int epc = rtck::format_elems_per_chunk(c->fmt);
    c->ldq = round_up(c->n_slopes, epc);
    c->n_chunks = (int32_t)(c->ldq / epc);
  }
  c->n_act = cfg->n_act;
  c->tiles_h = std::move(tiles);

  DeviceScope ds(c->device);
  auto bail = [&](hipError_t err2, const char *what) {
    const rtc_status st = hip_fail(nullptr, err2, what);
    rtc_destroy(c);
    return st;
  };
  if (ds.status != hipSuccess) return bail(ds.status, "rtc_init: hipSetDevice");
  if ((e = scratch_address(c->device, &c->d_scratch)) != hipSuccess) return bail(e, "rtc_init: hipGetSymbolAddress of the static scratch");
  int khz = 0;
  if ((e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device)) != hipSuccess)
    return bail(e, "rtc_init: wall clock rate");
  c->wall_khz = khz;
  int ncu = 0;
  if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device)) != hipSuccess)
    return bail(e, "rtc_init: compute-unit count");
  c->n_cu = ncu;
  const size_t s_bytes = (size_t)c->s_len * sizeof(float);
  const size_t t_bytes = (size_t)c->n_valid * sizeof(rtck::TileDesc);
  if ((e = hipMalloc(&c->d_tiles, t_bytes)) != hipSuccess ||
      (e = hipMalloc(&c->d_ref, s_bytes)) != hipSuccess ||
      (e = hipMalloc(&c->d_s, s_bytes)) != hipSuccess ||
      (e = hipMalloc(&c->d_state, c->n_act * sizeof(float))) != hipSuccess ||
      (e = hipMalloc(&c->d_part, (size_t)rtck::kMaxKSplit * c->n_act * sizeof(float))) != hipSuccess ||
      (e = hipMalloc(&c->d_sbuf, 4 * xchg_len_of(c->n_slopes) * sizeof(float))) != hipSuccess ||
      (e = hipMalloc(&c->d_sync, kSyncWords * sizeof(uint32_t))) != hipSuccess)
    return bail(e, "rtc_init: hipMalloc");
  if ((e = hipMemcpy(c->d_tiles, c->tiles_h.data(), t_bytes, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemset(c->d_ref, 0, s_bytes)) != hipSuccess ||
      (e = hipMemset(c->d_s, 0, s_bytes)) != hipSuccess ||
      (e = hipMemset(c->d_state, 0, c->n_act * sizeof(float))) != hipSuccess ||
      (e = hipMemset(c->d_sbuf, 0, 4 * xchg_len_of(c->n_slopes) * sizeof(float))) != hipSuccess ||
      (e = hipMemset(c->d_sync, 0, kSyncWords * sizeof(uint32_t))) != hipSuccess ||
      (e = hipDeviceSynchronize()) != hipSuccess)
    return bail(e, "rtc_init: device initialisation");
  c->err = "no error";
  *out = c;
  return RTC_OK;
}

rtc_status rtc_init(const rtc_config *cfg, rtc_ctx **out) {
  if (!cfg || !out) return fail(nullptr, RTC_E_ARG, "rtc_init: NULL config or output pointer");
  if (cfg->abi_version != RTC_ABI_VERSION)
    return fail(nullptr, RTC_E_ARG, "rtc_init: abi_version does not match RTC_ABI_VERSION");
  const rtc_wfs one{cfg->n_sub_x, cfg->n_sub_y, cfg->n_pix, cfg->subap_mask};
  return init_impl(cfg, &one, 1, "rtc_init", out);
}

rtc_status rtc_init_multi(const rtc_multi_config *mc, rtc_ctx **out) {
  if (!mc || !out) return fail(nullptr, RTC_E_ARG, "rtc_init_multi: NULL config or output pointer");
  rtc_config cfg{};
  cfg.abi_version = mc->abi_version;
  cfg.n_act = mc->n_act;
  cfg.thr_mode = mc->thr_mode;
  cfg.cm_dtype = mc->cm_dtype;
  cfg.gain = mc->gain;
  cfg.leak = mc->leak;
  cfg.cmd_min = mc->cmd_min;
  cfg.cmd_max = mc->cmd_max;
  cfg.device = mc->device;
  return init_impl(&cfg, mc->wfs, mc->n_wfs, "rtc_init_multi", out);
}

int64_t rtc_frame_elems(const rtc_ctx *c) { return c ? c->frame_elems : -1; }

// Validates and uploads dark, flat (frame-set layout), one threshold per sensor
// and the reference slopes.
static rtc_status load_calib_impl(rtc_ctx *c, const float *dark, const float *flat, const float *thr,
                                  const float *ref_slopes, const char *who) {
  auto err = [&](rtc_status st, const char *msg) { return fail(c, st, std::string(who) + ": " + msg); };
  if (!dark || !flat) return err(RTC_E_ARG, "NULL dark or flat map");
  for (size_t w = 0; w < c->wfs.size(); ++w) {
    if (!std::isfinite(thr[w])) return err(RTC_E_NONFINITE, "threshold not finite");
    if (thr[w] < 0.0f) return err(RTC_E_ARG, "threshold must be >= 0");
  }
  std::vector<float2> cal;
  std::vector<rtck::TileDesc> tiles = c->tiles_h;
  bool fast = true;                                // every dark admits the one-fma threshold decision
  try {
    cal.resize((size_t)c->calib_len);
  } catch (...) {
    return err(RTC_E_NOMEM, "host allocation failed");
  }
  for (size_t w = 0; w < c->wfs.size(); ++w) {
    const WfsInfo &wi = c->wfs[w];
    for (int32_t k = wi.tile_base; k < wi.tile_base + wi.n_tiles; ++k) {
      rtck::TileDesc &t = tiles[(size_t)k];
      t.thr = thr[w];
      const int n = t.n;
      for (int i = 0; i < n; ++i) {
        const int64_t base = (int64_t)t.off + (int64_t)i * t.pitch;
        for (int j = 0; j < n; ++j) {
          const float d = dark[base + j], f = flat[base + j];
          if (!std::isfinite(d) || !std::isfinite(f))
            return err(RTC_E_NONFINITE, "non-finite dark or flat value in an active subaperture");
          if (!dark_in_domain(d)) fast = false;
          cal[(size_t)t.calib_off + (size_t)i * n + j] = make_float2(d, f);
        }
      }
    }
  }
  std::vector<float> ref((size_t)c->s_len, 0.0f);
  if (ref_slopes) {
    for (int32_t i = 0; i < c->n_slopes; ++i) {
      if (!std::isfinite(ref_slopes[i])) return err(RTC_E_NONFINITE, "non-finite reference slope");
      ref[i] = ref_slopes[i];
    }
  }
  DeviceScope ds(c->device);
  if (ds.status != hipSuccess) return hip_fail(c, ds.status, "rtc_load_calib: hipSetDevice");
  float2 *d_cal = nullptr;
  hipError_t e = hipMalloc(&d_cal, cal.size() * sizeof(float2));
  if (e != hipSuccess) return hip_fail(c, e, "rtc_load_calib: hipMalloc");
  // frames already queued keep using the old buffers until the device is idle
  if ((e = hipDeviceSynchronize()) != hipSuccess ||
      (e = hipMemcpy(d_cal, cal.data(), cal.size() * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->d_ref, ref.data(), ref.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->d_tiles, tiles.data(), tiles.size() * sizeof(rtck::TileDesc), hipMemcpyHostToDevice)) !=
          hipSuccess) {
    (void)hipFree(d_cal);
    return hip_fail(c, e, "rtc_load_calib: upload");
  }
  dfree(c->d_calib);
  c->d_calib = d_cal;
  c->tiles_h = std::move(tiles);
  c->dark_fast = fast ? 1 : 0;
  c->calib_loaded = true;
  return RTC_OK;
}

rtc_status rtc_load_calib(rtc_ctx *c, const float *dark, const float *flat, float threshold,
                          const float *ref_slopes) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_load_calib: NULL context");
  std::vector<float> thr(c->wfs.size(), threshold);
  return load_calib_impl(c, dark, flat, thr.data(), ref_slopes, "rtc_load_calib");
}

rtc_status rtc_load_calib_multi(rtc_ctx *c, const float *dark, const float *flat, const float *thresholds,
                                const float *ref_slopes) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_load_calib_multi: NULL context");
  if (!thresholds) return fail(c, RTC_E_ARG, "rtc_load_calib_multi: NULL thresholds");
  return load_calib_impl(c, dark, flat, thresholds, ref_slopes, "rtc_load_calib_multi");
}

rtc_status rtc_load_cmat(rtc_ctx *c, const float *R, int32_t n_act, int32_t n_slopes, int64_t ld) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_load_cmat: NULL context");
  if (!R) return fail(c, RTC_E_ARG, "rtc_load_cmat: NULL matrix");
  if (n_act != c->n_act) return fail(c, RTC_E_ARG, "rtc_load_cmat: n_act differs from the configuration");
  if (n_slopes != c->n_slopes) return fail(c, RTC_E_ARG, "rtc_load_cmat: n_slopes must equal 2*n_valid");
  if (ld < n_slopes) return fail(c, RTC_E_ARG, "rtc_load_cmat: ld < n_slopes");
  for (int64_t r = 0; r < n_act; ++r) {
    const float *row = R + r * ld;
    for (int32_t j = 0; j < n_slopes; ++j)
      if (!std::isfinite(row[j])) return fail(c, RTC_E_NONFINITE, "rtc_load_cmat: non-finite matrix entry");
  }
  DeviceScope ds(c->device);
  if (ds.status != hipSuccess) return hip_fail(c, ds.status, "rtc_load_cmat: hipSetDevice");
  const FmtDesc &f = kFmt[c->fmt];
  const int64_t ldq = (c->fmt == RTC_CM_F32) ? c->ldr : c->ldq;
  const size_t bytes = (size_t)n_act * ldq * f.bytes;
  std::vector<uint8_t> codes;
  std::vector<float> scales;
  if (c->fmt != RTC_CM_F32) {
    try {
      codes.resize(bytes);
      scales.resize(n_act);
    } catch (...) {
      return fail(c, RTC_E_NOMEM, "rtc_load_cmat: host allocation failed");
    }
    encode_rows(c->fmt, R, n_act, n_slopes, ld, codes.data(), ldq, scales.data());
  }
  void *d_R = nullptr;
  float *d_sc = nullptr;
  hipError_t e = hipMalloc(&d_R, bytes);
  if (e == hipSuccess && c->fmt != RTC_CM_F32) e = hipMalloc(&d_sc, n_act * sizeof(float));
  if (e != hipSuccess) {
    if (d_R) (void)hipFree(d_R);
    return hip_fail(c, e, "rtc_load_cmat: hipMalloc");
  }
  if ((e = hipDeviceSynchronize()) == hipSuccess) {
    if (c->fmt == RTC_CM_F32) {
      if ((e = hipMemset(d_R, 0, bytes)) == hipSuccess)
        e = hipMemcpy2D(d_R, ldq * sizeof(float), R, ld * sizeof(float), n_slopes * sizeof(float), n_act,
                        hipMemcpyHostToDevice);
    } else {
      if ((e = hipMemcpy(d_R, codes.data(), bytes, hipMemcpyHostToDevice)) == hipSuccess)
        e = hipMemcpy(d_sc, scales.data(), n_act * sizeof(float), hipMemcpyHostToDevice);
    }
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    (void)hipFree(d_R);
    if (d_sc) (void)hipFree(d_sc);
    return hip_fail(c, e, "rtc_load_cmat: upload");
  }
  dfree(c->d_R);
  dfree(c->d_scales);
  c->d_R = d_R;
  c->d_scales = d_sc;
  c->cmat_loaded = true;
  ++c->cmat_gen;
  if (c->frame_mode == RTC_FRAMES_HORIZONTAL) return horiz_prepare(c, "rtc_load_cmat");
  return RTC_OK;
}

rtc_status rtc_encode_cmat(int32_t cm_dtype, const float *R, int32_t n_rows, int32_t n_cols, int64_t ld,
                           void *codes, float *scales) {
  if (cm_dtype != RTC_CM_F16 && cm_dtype != RTC_CM_BF16 && cm_dtype != RTC_CM_FP8E4M3)
    return fail(nullptr, RTC_E_ARG, "rtc_encode_cmat: cm_dtype must be F16, BF16 or FP8E4M3");
  if (!R || !codes || !scales) return fail(nullptr, RTC_E_ARG, "rtc_encode_cmat: NULL pointer");
  if (n_rows < 0 || n_cols < 0 || ld < n_cols) return fail(nullptr, RTC_E_ARG, "rtc_encode_cmat: bad sizes");
  for (int64_t r = 0; r < n_rows; ++r)
    for (int32_t j = 0; j < n_cols; ++j)
      if (!std::isfinite(R[r * ld + j])) return fail(nullptr, RTC_E_NONFINITE, "rtc_encode_cmat: non-finite entry");
  encode_rows(cm_dtype, R, n_rows, n_cols, ld, codes, n_cols, scales);
  return RTC_OK;
}

// Step (c)-(d) with the context's tuning; the row-block kernel falls back to
// the streamed kernel when the slope vector is too long for its registers.
static hipError_t launch_reconstruction(const rtc_ctx *c, rtck::MvmArgs ma, hipStream_t st) {
  const rtc_mvm_tuning &t = c->tuning;
  ma.R = c->fmt == RTC_CM_F32 ? static_cast<const float *>(c->d_R) : nullptr;
  ma.ldr = c->ldr;
  ma.Rq = c->d_R;
  ma.ldq_bytes = c->ldq * kFmt[c->fmt].bytes;
  ma.scales = c->d_scales;
  ma.fmt = c->fmt;
  ma.n_chunks = c->n_chunks;
  if (t.kernel == RTC_MVM_ROWBLOCK || c->fmt != RTC_CM_F32) {
    ma.k_split = 1;
    const int G = t.blocks > 0 ? t.blocks : c->n_cu;
    // slope vectors beyond 8 wavefronts' register slices: slope panels, sliced
    // as the persistent kernel slices them
    if (rtck::slice_chunks(c->n_chunks, 8) / 64 > rtck::mvm_block_max_kpl(c->fmt))
      return rtck::launch_mvm_panel(ma, G, st);
    return rtck::launch_mvm_block(ma, G, t.waves, t.rows_per_wave, st);
  }
  return rtck::launch_mvm_integrate(ma, nullptr, st);
}

// Calibration arguments of one frame set (outputs left for the caller to set).
// Largest float2 count of one workgroup's (dark, flat) blocks when G
// workgroups share the subapertures of a persistent launch (the blocks are
// contiguous in subaperture order).
static int32_t calib_span(const rtc_ctx *c, int G) {
  int64_t span = 0;
  const int64_t n = c->n_valid;
  for (int b = 0; b < G; ++b) {
    const int64_t k0 = (int64_t)b * n / G, k1 = (int64_t)(b + 1) * n / G;
    if (k1 <= k0) continue;
    const int64_t lo = c->tiles_h[(size_t)k0].calib_off;
    const int64_t hi = k1 < n ? (int64_t)c->tiles_h[(size_t)k1].calib_off : c->calib_len;
    span = std::max(span, hi - lo);
  }
  return span > INT32_MAX ? 0 : (int32_t)span;
}

static rtck::CalibArgs calib_args(const rtc_ctx *c, const uint16_t *pix) {
  rtck::CalibArgs ca{};
  ca.pix = pix;
  ca.tiles = c->d_tiles;
  ca.calib = c->d_calib;
  ca.n_valid = c->n_valid;
  ca.max_n = c->max_n;
  ca.pairs = c->pairs;
  ca.mode = c->cfg.thr_mode;
  ca.dark_fast = c->dark_fast;
  ca.ref = c->d_ref;
  return ca;
}

static FrameScratch ctx_scratch(const rtc_ctx *c) { return FrameScratch{c->d_s, c->d_part, c->d_sync}; }

static rtc_status enqueue_frame(rtc_ctx *c, const FrameScratch &fs, const uint16_t *pix, float *cmd, float *slopes,
                                float *recon, int32_t *counts, uint64_t *ts, hipStream_t st, const char *who,
                                rtcx::SlopeStep step = nullptr, void *step_arg = nullptr) {
  rtck::CalibArgs ca = calib_args(c, pix);
  ca.s_int = fs.s;
  ca.s_user = slopes;
  ca.counts = counts;
  ca.ts_start = ts;
  hipError_t e = rtck::launch_calib_cog(ca, st);
  if (e != hipSuccess) return hip_fail(c, e, who);
  const float *s_use = fs.s;
  if (step != nullptr && (e = step(step_arg, fs.s, c->d_state, &s_use, st)) != hipSuccess) return hip_fail(c, e, who);
  rtck::MvmArgs ma{};
  ma.n_act = c->n_act;
  ma.n_s4 = c->n_s4;
  ma.s = s_use;
  ma.k_split = c->tuning.k_split;
  ma.rows_per_wave = c->tuning.rows_per_wave;
  ma.unroll = c->tuning.unroll;
  ma.part = fs.part;
  ma.state = c->d_state;
  ma.cmd = cmd;
  ma.recon = recon;
  ma.gain = c->cfg.gain;
  ma.leak = c->cfg.leak;
  ma.cmd_min = c->cfg.cmd_min;
  ma.cmd_max = c->cfg.cmd_max;
  ma.sync = fs.sync;
  ma.ts_end = ts ? ts + 1 : nullptr;
  e = launch_reconstruction(c, ma, st);
  if (e != hipSuccess) return hip_fail(c, e, who);
  return RTC_OK;
}

rtc_status rtc_frame(rtc_ctx *c, const uint16_t *d_pixels, float *d_cmd, float *d_slopes, float *d_recon,
                     int32_t *d_counts, void *hip_stream) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_frame: NULL context");
  if (!c->calib_loaded || !c->cmat_loaded)
    return fail(c, RTC_E_STATE, "rtc_frame: load the calibration and the control matrix first");
  if (c->state_invalid) return fail(c, RTC_E_STATE, "rtc_frame: " STATE_INVALID_MSG);
  if (!d_pixels || !d_cmd) return fail(c, RTC_E_ARG, "rtc_frame: NULL pixels or cmd");
  DeviceScope ds(c->device);
  if (ds.status != hipSuccess) return hip_fail(c, ds.status, "rtc_frame: hipSetDevice");
  return enqueue_frame(c, ctx_scratch(c), d_pixels, d_cmd, d_slopes, d_recon, d_counts, nullptr,
                       static_cast<hipStream_t>(hip_stream), "rtc_frame: launch");
}

// Arguments of a persistent launch (either split) of n_frames frame sets.
static rtck::PersistArgs persist_args(const rtc_ctx *c, int32_t n_frames, const uint16_t *d_pixels,
                                      int64_t frame_stride, float *d_cmd, float *d_slopes, float *d_recon,
                                      int32_t *d_counts, uint64_t *d_ts) {
  rtck::PersistArgs p{};
  p.cal = calib_args(c, d_pixels);
  p.cal.s_user = d_slopes;
  p.cal.counts = d_counts;
  p.frame_stride = frame_stride;
  p.n_frames = n_frames;
  p.vec = (c->pairs && (frame_stride & 1) == 0 && (reinterpret_cast<uintptr_t>(d_pixels) & 3) == 0) ? 1 : 0;
  p.sbuf = c->d_sbuf;
  p.s_len = (int32_t)xchg_len_of(c->n_slopes);
  p.cal.xchg_epc = rtck::format_elems_per_chunk(c->fmt);
  rtck::MvmArgs &ma = p.mvm;
  ma.Rq = c->d_R;
  ma.ldq_bytes = c->ldq * kFmt[c->fmt].bytes;
  ma.scales = c->d_scales;
  ma.fmt = c->fmt;
  ma.n_chunks = c->n_chunks;
  ma.n_act = c->n_act;
  ma.state = c->d_state;
  ma.cmd = d_cmd;
  ma.recon = d_recon;
  ma.gain = c->cfg.gain;
  ma.leak = c->cfg.leak;
  ma.cmd_min = c->cfg.cmd_min;
  ma.cmd_max = c->cfg.cmd_max;
  p.bar = c->d_sync + rtck::sync_layout::kBarBase;
  p.abort_flag = c->d_sync + rtck::sync_layout::kAbort;
  p.sticky = c->d_sync + rtck::sync_layout::kSticky;
  p.spin_limit = c->spin_limit;
  p.ts = d_ts;
  p.trace = c->d_trace;
  p.trace_frames = c->trace_frames;
  p.trace_groups = c->trace_groups;
  return p;
}

// Shape of the horizontal frames for this context: subapertures per workgroup
// (nch), rows per owner (nrt) and 16-byte chunks per row slot (nq); false with
// the reason when the built kernels do not cover it.
static bool horiz_shape(const rtc_ctx *c, int32_t *nch, int32_t *nrt, int32_t *nq, std::string *why) {
  const int G = rtck::kHoriz;
  if (c->n_cu < G) {
    *why = "the horizontal split needs 256 compute units";
    return false;
  }
  if (c->max_n > 16 || (c->fmt == RTC_CM_F32 && c->max_n > 10 && (c->n_valid + G - 1) / G > 4)) {
    *why = "subapertures wider than the horizontal kernels' tiles (16 pixels; 10 for wide FP32 slabs)";
    return false;
  }
  if (!c->pairs) {
    *why = "the horizontal kernels read 4-byte pixel pairs (even tile widths and frame layout)";
    return false;
  }
  const int32_t ch = (c->n_valid + G - 1) / G;
  const int32_t q = rtck::horiz_chunks(c->fmt, ch);
  if (q == 0) {
    *why = "more than 32 slope columns per workgroup";
    return false;
  }
  const int32_t rows = (c->n_act + G - 1) / G;
  if (rows > rtck::horiz_max_rows(c->fmt, q)) {
    *why = "more actuator rows per workgroup than the horizontal kernels hold on chip";
    return false;
  }
  *nch = ch;
  *nrt = rows;
  *nq = q;
  return true;
}

// Builds the horizontal layout of the loaded matrix and zeroes the message
// buffer (synchronous); a no-op without a matrix.
static rtc_status horiz_prepare(rtc_ctx *c, const char *who) {
  if (!c->cmat_loaded) return RTC_OK;
  int32_t nch = 0, nrt = 0, nq = 0;
  std::string why;
  if (!horiz_shape(c, &nch, &nrt, &nq, &why)) return fail(c, RTC_E_UNSUPPORTED, std::string(who) + ": " + why);
  const int G = rtck::kHoriz;
  const int64_t chunks = rtck::horiz_layout_chunks(G, nrt, nq);
  const size_t xfloats = (size_t)2 * G * G * rtck::kHorizMsg;
  hipError_t e = hipSuccess;
  if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(c, e, who);
  if (c->hm_chunks != chunks) {
    dfree(c->d_hm);
    c->hm_chunks = 0;
    c->h_gen = 0;
    if ((e = hipMalloc(&c->d_hm, (size_t)chunks * sizeof(uint4))) != hipSuccess) return hip_fail(c, e, who);
    c->hm_chunks = chunks;
  }
  if (!c->d_xbuf && (e = hipMalloc(&c->d_xbuf, xfloats * sizeof(float))) != hipSuccess) return hip_fail(c, e, who);
  if ((e = rtck::launch_horiz_layout(c->d_R, c->ldq * kFmt[c->fmt].bytes, c->fmt, c->d_tiles, c->n_valid, c->n_act,
                                     G, nch, nrt, nq, c->d_hm, nullptr)) != hipSuccess ||
      (e = rtck::launch_fill_zero(c->d_xbuf, (int64_t)xfloats, nullptr)) != hipSuccess ||
      (e = hipDeviceSynchronize()) != hipSuccess)
    return hip_fail(c, e, who);
  c->h_gen = c->cmat_gen;
  c->h_nch = nch;
  c->h_nrt = nrt;
  c->h_nq = nq;
  return RTC_OK;
}

rtc_status rtc_frame_batch(rtc_ctx *c, int32_t n_frames, const uint16_t *d_pixels, int64_t frame_stride,
                           float *d_cmd, float *d_slopes, float *d_recon, int32_t *d_counts, uint64_t *d_ts,
                           void *hip_stream) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_frame_batch: NULL context");
  if (!c->calib_loaded || !c->cmat_loaded)
    return fail(c, RTC_E_STATE, "rtc_frame_batch: load the calibration and the control matrix first");
  if (c->state_invalid) return fail(c, RTC_E_STATE, "rtc_frame_batch: " STATE_INVALID_MSG);
  if (n_frames < 0) return fail(c, RTC_E_ARG, "rtc_frame_batch: n_frames < 0");
  if (n_frames == 0) return RTC_OK;
  if (!d_pixels || !d_cmd) return fail(c, RTC_E_ARG, "rtc_frame_batch: NULL pixels or cmd");
  if (frame_stride < c->frame_elems)
    return fail(c, RTC_E_ARG, "rtc_frame_batch: frame_stride shorter than a frame");
  DeviceScope ds(c->device);
  if (ds.status != hipSuccess) return hip_fail(c, ds.status, "rtc_frame_batch: hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (c->frame_mode == RTC_FRAMES_HORIZONTAL) {
    rtc_status hs = c->h_gen == c->cmat_gen ? RTC_OK : horiz_prepare(c, "rtc_frame_batch");
    if (hs != RTC_OK) return hs;
    rtck::HorizArgs h{};
    h.p = persist_args(c, n_frames, d_pixels, frame_stride, d_cmd, d_slopes, d_recon, d_counts, d_ts);
    h.hm = c->d_hm;
    h.xbuf = c->d_xbuf;
    h.nch = c->h_nch;
    h.nrt = c->h_nrt;
    hipError_t e = rtck::launch_horizontal(h, st);
    if (e == hipSuccess) return RTC_OK;
    if (e != hipErrorInvalidValue && e != hipErrorCooperativeLaunchTooLarge)
      return hip_fail(c, e, "rtc_frame_batch: horizontal launch");
    (void)hipGetLastError();   // unsupported shape or frames: one launch pair per frame
  }
  if (c->frame_mode == RTC_FRAMES_PERSISTENT) {
    rtck::PersistArgs p = persist_args(c, n_frames, d_pixels, frame_stride, d_cmd, d_slopes, d_recon, d_counts, d_ts);
    const int blocks = c->tuning.blocks > 0 ? c->tuning.blocks : c->n_cu;
    const int G = rtck::frames_grid(blocks, c->n_act);
    p.calib_span = calib_span(c, G);
    if (c->split_G > 0 && c->split_G == G) {
      p.row_start = c->d_row_start;
      p.row_max = c->split_max;
    }
    hipError_t e = rtck::launch_frames(p, blocks, c->tuning.rows_per_wave, st);
    if (e == hipSuccess) return RTC_OK;
    if (e != hipErrorInvalidValue && e != hipErrorCooperativeLaunchTooLarge)
      return hip_fail(c, e, "rtc_frame_batch: persistent launch");
    (void)hipGetLastError();   // unsupported shape: fall through to one launch pair per frame
  }
  const FrameScratch fs = ctx_scratch(c);
  for (int32_t f = 0; f < n_frames; ++f) {
    rtc_status s = enqueue_frame(c, fs, d_pixels + (int64_t)f * frame_stride, d_cmd + (int64_t)f * c->n_act,
                                 d_slopes ? d_slopes + (int64_t)f * c->n_slopes : nullptr,
                                 d_recon ? d_recon + (int64_t)f * c->n_act : nullptr,
                                 d_counts ? d_counts + (int64_t)f * c->n_valid : nullptr,
                                 d_ts ? d_ts + 2 * (int64_t)f : nullptr, st, "rtc_frame_batch: launch");
    if (s != RTC_OK) return s;
  }
  return RTC_OK;
}

rtc_status rtc_frame_batch_noalloc(rtc_ctx *c, int32_t n_frames, const uint16_t *d_pixels, int64_t frame_stride,
                                   float *d_cmd, float *d_slopes, float *d_recon, int32_t *d_counts, uint64_t *d_ts,
                                   void *hip_stream) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_frame_batch_noalloc: NULL context");
  if (!c->calib_loaded || !c->cmat_loaded)
    return fail(c, RTC_E_STATE, "rtc_frame_batch_noalloc: load the calibration and the control matrix first");
  if (c->state_invalid) return fail(c, RTC_E_STATE, "rtc_frame_batch_noalloc: " STATE_INVALID_MSG);
  if (n_frames < 0) return fail(c, RTC_E_ARG, "rtc_frame_batch_noalloc: n_frames < 0");
  if (n_frames == 0) return RTC_OK;
  if (!d_pixels || !d_cmd) return fail(c, RTC_E_ARG, "rtc_frame_batch_noalloc: NULL pixels or cmd");
  if (frame_stride < c->frame_elems)
    return fail(c, RTC_E_ARG, "rtc_frame_batch_noalloc: frame_stride shorter than a frame");
  if (!c->d_scratch)
    return fail(c, RTC_E_UNSUPPORTED, "rtc_frame_batch_noalloc: no static scratch for device ordinals above 63");
  const ScratchLayout L = scratch_layout(c);
  if (L.words > kScratchWords)
    return fail(c, RTC_E_UNSUPPORTED,
                "rtc_frame_batch_noalloc: this context needs " + std::to_string(L.words * 4) +
                    " bytes of static scratch (2 (2 n_valid rounded up to 1024) + (2 n_valid rounded up to 16) + "
                    "k_split n_act floats plus 152 KiB of barrier words); the limit is " +
                    std::to_string(kScratchWords * 4) + " bytes");
  DeviceScope ds(c->device);
  if (ds.status != hipSuccess) return hip_fail(c, ds.status, "rtc_frame_batch_noalloc: hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  uint32_t *const base = c->d_scratch;
  // the counter and abort words, both slope buffers (their padding is read)
  hipError_t e = rtck::launch_fill_zero(reinterpret_cast<float *>(base), L.zero_words, st);
  if (e != hipSuccess) return hip_fail(c, e, "rtc_frame_batch_noalloc: scratch clear");
  // horizontal mode needs its 16.8 MB message buffer: the row split runs instead
  if (c->frame_mode != RTC_FRAMES_PER_LAUNCH) {
    rtck::PersistArgs p = persist_args(c, n_frames, d_pixels, frame_stride, d_cmd, d_slopes, d_recon, d_counts, d_ts);
    p.sbuf = reinterpret_cast<float *>(base + L.sbuf);
    p.bar = base + L.bar;
    p.abort_flag = base + 1;
    // p.sticky stays the context's word, which rtc_sync_check reads
    const int blocks = c->tuning.blocks > 0 ? c->tuning.blocks : c->n_cu;
    const int G = rtck::frames_grid(blocks, c->n_act);
    p.calib_span = calib_span(c, G);
    if (c->split_G > 0 && c->split_G == G) {
      p.row_start = c->d_row_start;
      p.row_max = c->split_max;
    }
    e = rtck::launch_frames(p, blocks, c->tuning.rows_per_wave, st);
    if (e == hipSuccess) return RTC_OK;
    if (e != hipErrorInvalidValue && e != hipErrorCooperativeLaunchTooLarge)
      return hip_fail(c, e, "rtc_frame_batch_noalloc: persistent launch");
    (void)hipGetLastError();
  }
  const FrameScratch fs{reinterpret_cast<float *>(base + L.s), reinterpret_cast<float *>(base + L.part), base};
  for (int32_t f = 0; f < n_frames; ++f) {
    rtc_status s = enqueue_frame(c, fs, d_pixels + (int64_t)f * frame_stride, d_cmd + (int64_t)f * c->n_act,
                                 d_slopes ? d_slopes + (int64_t)f * c->n_slopes : nullptr,
                                 d_recon ? d_recon + (int64_t)f * c->n_act : nullptr,
                                 d_counts ? d_counts + (int64_t)f * c->n_valid : nullptr,
                                 d_ts ? d_ts + 2 * (int64_t)f : nullptr, st, "rtc_frame_batch_noalloc: launch");
    if (s != RTC_OK) return s;
  }
  return RTC_OK;
}

rtc_status rtc_paced_batch(rtc_ctx *c, int32_t n_frames, const uint16_t *d_pixels, int64_t frame_stride,
                           float *d_cmd, float *d_slopes, float *d_recon, int32_t *d_counts, uint64_t *d_ts,
                           double period_us, int64_t *h_release_ns, int64_t *h_done_ns, void *hip_stream) {
  // host times from CLOCK_MONOTONIC_RAW (not slewed by time adjustment), in ns
  auto now_ns = []() -> int64_t {
    timespec t;
    clock_gettime(CLOCK_MONOTONIC_RAW, &t);
    return (int64_t)t.tv_sec * 1000000000 + t.tv_nsec;
  };
  const char *who = "rtc_paced_batch";
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_paced_batch: NULL context");
  if (!c->calib_loaded || !c->cmat_loaded)
    return fail(c, RTC_E_STATE, "rtc_paced_batch: load the calibration and the control matrix first");
  if (c->state_invalid) return fail(c, RTC_E_STATE, "rtc_paced_batch: " STATE_INVALID_MSG);
  if (c->frame_mode != RTC_FRAMES_PERSISTENT)
    return fail(c, RTC_E_STATE, "rtc_paced_batch: needs RTC_FRAMES_PERSISTENT");
  if (n_frames < 0) return fail(c, RTC_E_ARG, "rtc_paced_batch: n_frames < 0");
  if (n_frames == 0) return RTC_OK;
  if (!d_pixels || !d_cmd) return fail(c, RTC_E_ARG, "rtc_paced_batch: NULL pixels or cmd");
  if (frame_stride < c->frame_elems) return fail(c, RTC_E_ARG, "rtc_paced_batch: frame_stride shorter than a frame");
  if (!(period_us > 0.0) || period_us > 1e7) return fail(c, RTC_E_ARG, "rtc_paced_batch: period_us must be in (0, 1e7]");
  if (!c->dark_fast)
    return fail(c, RTC_E_UNSUPPORTED, "rtc_paced_batch: the persistent kernel needs darks in {0} U [2^-13, 2^24)");
  DeviceScope ds(c->device);
  if (ds.status != hipSuccess) return hip_fail(c, ds.status, who);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  hipError_t e = hipSuccess;
  if (!c->h_trig) {
    void *h = nullptr;
    if ((e = hipHostMalloc(&h, 256, hipHostMallocCoherent | hipHostMallocMapped)) != hipSuccess)
      return hip_fail(c, e, "rtc_paced_batch: hipHostMalloc of the trigger words");
    c->h_trig = static_cast<uint32_t *>(h);
    __atomic_store_n(c->h_trig, c->trig_base, __ATOMIC_RELEASE);
    __atomic_store_n(c->h_trig + 32, c->trig_base, __ATOMIC_RELEASE);
  }
  void *d_trig = nullptr;
  if ((e = hipHostGetDevicePointer(&d_trig, c->h_trig, 0)) != hipSuccess)
    return hip_fail(c, e, "rtc_paced_batch: hipHostGetDevicePointer");
  rtck::PersistArgs p = persist_args(c, n_frames, d_pixels, frame_stride, d_cmd, d_slopes, d_recon, d_counts, d_ts);
  const uint32_t base = c->trig_base;
  p.trig_release = static_cast<const uint32_t *>(d_trig);
  p.trig_done = static_cast<uint32_t *>(d_trig) + 32;
  p.trig_base = base;
  const int blocks = c->tuning.blocks > 0 ? c->tuning.blocks : c->n_cu;
  const int G = rtck::frames_grid(blocks, c->n_act);
  p.calib_span = calib_span(c, G);
  if (c->split_G > 0 && c->split_G == G) {
    p.row_start = c->d_row_start;
    p.row_max = c->split_max;
  }
  e = rtck::launch_frames(p, blocks, c->tuning.rows_per_wave, st);
  if (e == hipErrorInvalidValue) {
    (void)hipGetLastError();
    return fail(c, RTC_E_UNSUPPORTED, "rtc_paced_batch: shape not covered by the triggered persistent kernel "
                                      "(tiles of up to 16 pixels, slope vectors without panels, slabs within "
                                      "the persistent limits)");
  }
  if (e != hipSuccess) return hip_fail(c, e, "rtc_paced_batch: persistent launch");
  // frames released from here on belong to this batch, whatever happens below
  c->trig_base = base + (uint32_t)n_frames;
  volatile uint32_t *release = c->h_trig;
  const volatile uint32_t *done = c->h_trig + 32;
  const int64_t period = std::llround(period_us * 1e3);
  const int64_t t0 = now_ns() + period;
  // a frame not done within 100 periods (at least 100 ms) fails the batch
  const int64_t limit = std::max<int64_t>(100000000, 100 * period);
  std::string late;
  for (int32_t k = 0; k < n_frames && late.empty(); ++k) {
    const int64_t due = t0 + (int64_t)k * period;
    while (now_ns() < due) {
    }
    const uint32_t v = base + (uint32_t)k + 1u;
    __atomic_store_n(const_cast<uint32_t *>(release), v, __ATOMIC_RELEASE);
    const int64_t t_rel = now_ns();
    if (h_release_ns) h_release_ns[k] = t_rel - t0;
    for (uint64_t spin = 0;; ++spin) {
      if ((int32_t)(__atomic_load_n(const_cast<uint32_t *>(done), __ATOMIC_ACQUIRE) - v) >= 0) break;
      if ((spin & 4095) == 4095 && now_ns() - t_rel > limit) {
        late = "rtc_paced_batch: frame " + std::to_string(k) + " was not done within " +
               std::to_string(limit / 1000000) + " ms";
        break;
      }
    }
    if (h_done_ns && late.empty()) h_done_ns[k] = now_ns() - t0;
  }
  // release whatever is left (a failed batch then winds down at once) and wait
  __atomic_store_n(const_cast<uint32_t *>(release), c->trig_base, __ATOMIC_RELEASE);
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(c, e, "rtc_paced_batch: synchronise");
  if (!late.empty()) return fail(c, RTC_E_DEVICE, late);
  return RTC_OK;
}

rtc_status rtc_graph_capture(rtc_ctx *c, int32_t n_frames, const uint16_t *d_pixels, int64_t frame_stride,
                             float *d_cmd, float *d_slopes, float *d_recon, int32_t *d_counts, uint64_t *d_ts) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_graph_capture: NULL context");
  if (n_frames < 1) return fail(c, RTC_E_ARG, "rtc_graph_capture: n_frames must be >= 1");
  DeviceScope ds(c->device);
  if (ds.status != hipSuccess) return hip_fail(c, ds.status, "rtc_graph_capture: hipSetDevice");
  hipStream_t s = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(c, e, "rtc_graph_capture: stream");
  if ((e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed)) != hipSuccess) {
    (void)hipStreamDestroy(s);
    return hip_fail(c, e, "rtc_graph_capture: begin capture");
  }
  const rtc_status st = rtc_frame_batch(c, n_frames, d_pixels, frame_stride, d_cmd, d_slopes, d_recon, d_counts,
                                        d_ts, s);
  hipGraph_t g = nullptr;
  const hipError_t e_end = hipStreamEndCapture(s, &g);
  hipGraphExec_t ex = nullptr;
  hipError_t e_inst = hipSuccess;
  if (st == RTC_OK && e_end == hipSuccess && g) e_inst = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(s);
  (void)hipGetLastError();
  if (st == RTC_E_ARG || st == RTC_E_STATE) return st;      // the call itself was invalid (message set)
  if (st != RTC_OK || e_end != hipSuccess || e_inst != hipSuccess || !ex) {
    if (ex) (void)hipGraphExecDestroy(ex);
    const hipError_t why = e_end != hipSuccess ? e_end : e_inst;
    return fail(c, RTC_E_UNSUPPORTED, std::string("rtc_graph_capture: the runtime did not record this frame mode (") +
                                           (st != RTC_OK ? c->err : std::string(hipGetErrorName(why))) + ")");
  }
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  c->graph = ex;
  return RTC_OK;
}

rtc_status rtc_graph_launch(rtc_ctx *c, void *hip_stream) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_graph_launch: NULL context");
  if (!c->graph) return fail(c, RTC_E_STATE, "rtc_graph_launch: no recorded graph");
  if (c->state_invalid) return fail(c, RTC_E_STATE, "rtc_graph_launch: " STATE_INVALID_MSG);
  DeviceScope ds(c->device);
  if (ds.status != hipSuccess) return hip_fail(c, ds.status, "rtc_graph_launch: hipSetDevice");
  const hipError_t e = hipGraphLaunch(c->graph, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? RTC_OK : hip_fail(c, e, "rtc_graph_launch");
}

rtc_status rtc_autotune(rtc_ctx *c, int32_t n_frames, const uint16_t *d_pixels, int64_t frame_stride,
                        float *d_cmd, rtc_tune_result *results, int32_t max_results, int32_t *n_results,
                        void *hip_stream) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_autotune: NULL context");
  if (n_frames < 1) return fail(c, RTC_E_ARG, "rtc_autotune: n_frames must be >= 1");
  if (!c->calib_loaded || !c->cmat_loaded)
    return fail(c, RTC_E_STATE, "rtc_autotune: load the calibration and the control matrix first");
  if (!d_pixels || !d_cmd) return fail(c, RTC_E_ARG, "rtc_autotune: NULL pixels or cmd");
  if (frame_stride < c->frame_elems) return fail(c, RTC_E_ARG, "rtc_autotune: frame_stride shorter than a frame");
  DeviceScope ds(c->device);
  if (ds.status != hipSuccess) return hip_fail(c, ds.status, "rtc_autotune: hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  std::vector<rtc_tune_result> cand;
  const int ncu = c->n_cu;
  auto add = [&](int mode, int kernel, int ks, int rpw, int unroll, int blocks, int waves) {
    rtc_tune_result r{};
    r.frame_mode = mode;
    r.tuning = rtc_mvm_tuning{kernel, ks, rpw, unroll, blocks, waves};
    r.us_per_frame = -1.0f;
    cand.push_back(r);
  };
  add(RTC_FRAMES_PERSISTENT, RTC_MVM_ROWBLOCK, 1, 2, 4, ncu, 8);
  add(RTC_FRAMES_PERSISTENT, RTC_MVM_ROWBLOCK, 1, 2, 4, ncu * 3 / 4, 8);
  for (int waves : {8, 16})
    for (int rb : {1, 2, 4})
      for (int mul : {1, 2}) add(RTC_FRAMES_PER_LAUNCH, RTC_MVM_ROWBLOCK, 1, rb, 4, ncu * mul, waves);
  if (c->fmt == RTC_CM_F32)
    for (int ks : {1, 2, 4}) add(RTC_FRAMES_PER_LAUNCH, RTC_MVM_STREAMED, ks, 2, 4, 0, 8);

  std::vector<float> saved((size_t)c->n_act);
  rtc_status s = rtc_get_state(c, saved.data());
  if (s != RTC_OK) return s;
  const int32_t mode0 = c->frame_mode;
  const rtc_mvm_tuning tune0 = c->tuning;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(c, e, "rtc_autotune: events");
  }
  const int32_t warm = n_frames / 4 + 1;
  int best = -1;
  for (size_t i = 0; i < cand.size(); ++i) {
    rtc_tune_result &r = cand[i];
    c->frame_mode = r.frame_mode;
    c->tuning = r.tuning;
    bool ok = rtc_frame_batch(c, std::min(warm, n_frames), d_pixels, frame_stride, d_cmd, nullptr, nullptr,
                              nullptr, nullptr, st) == RTC_OK;
    ok = ok && hipEventRecord(e0, st) == hipSuccess;
    ok = ok && rtc_frame_batch(c, n_frames, d_pixels, frame_stride, d_cmd, nullptr, nullptr, nullptr, nullptr,
                               st) == RTC_OK;
    ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float ms = 0.0f;
    ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    uint32_t aborted = 0;
    ok = ok && hipMemcpy(&aborted, c->d_sync + rtck::sync_layout::kSticky, sizeof(aborted),
                         hipMemcpyDeviceToHost) == hipSuccess;
    if (aborted) (void)hipMemset(c->d_sync + rtck::sync_layout::kSticky, 0, sizeof(uint32_t));
    ok = ok && aborted == 0;
    if (ok) {
      r.us_per_frame = ms * 1000.0f / (float)n_frames;
      if (best < 0 || r.us_per_frame < cand[(size_t)best].us_per_frame) best = (int)i;
    }
    (void)hipGetLastError();
    (void)hipDeviceSynchronize();
    if ((s = rtc_set_state(c, saved.data())) != RTC_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != RTC_OK || best < 0) {
    c->frame_mode = mode0;
    c->tuning = tune0;
    return s != RTC_OK ? s : fail(c, RTC_E_DEVICE, "rtc_autotune: no candidate ran");
  }
  c->frame_mode = cand[(size_t)best].frame_mode;
  c->tuning = cand[(size_t)best].tuning;
  if (results)
    for (int32_t i = 0; i < max_results && (size_t)i < cand.size(); ++i) results[i] = cand[(size_t)i];
  if (n_results) *n_results = (int32_t)cand.size();
  return RTC_OK;
}

rtc_status rtc_set_row_split(rtc_ctx *c, int32_t G, const int32_t *row_start) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_set_row_split: NULL context");
  if (G < 0 || G > rtck::sync_layout::kMaxGroups)
    return fail(c, RTC_E_ARG, "rtc_set_row_split: G must be in [0, 1024]");
  int32_t most = 0;
  if (G > 0 && row_start) {
    if (row_start[0] != 0 || row_start[G] != c->n_act)
      return fail(c, RTC_E_ARG, "rtc_set_row_split: row_start[0] must be 0 and row_start[G] n_act");
    for (int32_t b = 0; b < G; ++b) {
      const int32_t n = row_start[b + 1] - row_start[b];
      if (n < 1 || n > 512) return fail(c, RTC_E_ARG, "rtc_set_row_split: every share must hold 1 to 512 rows");
      most = std::max(most, n);
    }
  }
  DeviceScope ds(c->device);
  if (ds.status != hipSuccess) return hip_fail(c, ds.status, "rtc_set_row_split: hipSetDevice");
  // batches in flight may read the current split
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(c, e, "rtc_set_row_split: synchronize");
  if (c->graph) {                                  // recorded with the old launch shape
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  if (G == 0 || !row_start) {
    c->split_G = 0;
    c->split_max = 0;
    c->split_h.clear();
    return RTC_OK;
  }
  if (!c->d_row_start) {
    e = hipMalloc(&c->d_row_start, sizeof(int32_t) * (rtck::sync_layout::kMaxGroups + 1));
    if (e != hipSuccess) {
      c->d_row_start = nullptr;
      return hip_fail(c, e, "rtc_set_row_split: hipMalloc");
    }
  }
  e = hipMemcpy(c->d_row_start, row_start, sizeof(int32_t) * ((size_t)G + 1), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    c->split_G = 0;
    return hip_fail(c, e, "rtc_set_row_split: copy");
  }
  c->split_h.assign(row_start, row_start + G + 1);
  c->split_G = G;
  c->split_max = most;
  return RTC_OK;
}

rtc_status rtc_get_row_split(const rtc_ctx *c, int32_t *G, int32_t *row_start, int32_t capacity) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_get_row_split: NULL context");
  if (G) *G = c->split_G;
  if (row_start && c->split_G > 0) {
    if (capacity < c->split_G + 1) return fail(const_cast<rtc_ctx *>(c), RTC_E_ARG, "rtc_get_row_split: capacity < G + 1");
    std::copy(c->split_h.begin(), c->split_h.end(), row_start);
  }
  return RTC_OK;
}

// Shares of n rows in proportion to w (all > 0): floor of each plus the
// largest remainders (ties to the lower index), each share in [1, cap].
static std::vector<int32_t> proportional_split(const std::vector<double> &w, int32_t n, int32_t cap) {
  const size_t G = w.size();
  double tot = 0.0;
  for (double x : w) tot += x;
  std::vector<int32_t> cnt(G, 1);
  int32_t left = n - (int32_t)G;                   // one row each first
  std::vector<std::pair<double, size_t>> rem;
  for (size_t b = 0; b < G; ++b) {
    const double x = (double)left * w[b] / tot;
    const int32_t f = (int32_t)std::floor(x);
    cnt[b] += f;
    rem.push_back({x - f, b});
  }
  int32_t given = 0;
  for (int32_t x : cnt) given += x;
  std::stable_sort(rem.begin(), rem.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
  for (size_t i = 0; given < n && i < rem.size(); ++i, ++given) ++cnt[rem[i].second];
  // cap: move the excess to the workgroups with the most room, in index order
  for (size_t b = 0; b < G; ++b)
    while (cnt[b] > cap) {
      size_t best = b;
      for (size_t j = 0; j < G; ++j)
        if (cnt[j] < cnt[best]) best = j;
      if (cnt[best] >= cap) break;
      --cnt[b];
      ++cnt[best];
    }
  std::vector<int32_t> start(G + 1, 0);
  for (size_t b = 0; b < G; ++b) start[b + 1] = start[b] + cnt[b];
  return start;
}

rtc_status rtc_balance_rows(rtc_ctx *c, int32_t n_frames, const uint16_t *d_pixels, int64_t frame_stride,
                            float *d_cmd, float *us_equal, float *us_split, void *hip_stream) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_balance_rows: NULL context");
  if (n_frames < 4) return fail(c, RTC_E_ARG, "rtc_balance_rows: n_frames must be >= 4");
  if (!c->calib_loaded || !c->cmat_loaded)
    return fail(c, RTC_E_STATE, "rtc_balance_rows: load the calibration and the control matrix first");
  if (c->frame_mode != RTC_FRAMES_PERSISTENT)
    return fail(c, RTC_E_STATE, "rtc_balance_rows: the context is not in the persistent frame mode");
  if (!d_pixels || !d_cmd) return fail(c, RTC_E_ARG, "rtc_balance_rows: NULL pixels or cmd");
  if (frame_stride < c->frame_elems) return fail(c, RTC_E_ARG, "rtc_balance_rows: frame_stride shorter than a frame");
  DeviceScope ds(c->device);
  if (ds.status != hipSuccess) return hip_fail(c, ds.status, "rtc_balance_rows: hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int G = rtck::frames_grid(c->tuning.blocks > 0 ? c->tuning.blocks : c->n_cu, c->n_act);
  if (G > rtck::sync_layout::kMaxGroups) return fail(c, RTC_E_STATE, "rtc_balance_rows: grid too large");

  std::vector<float> saved((size_t)c->n_act);
  rtc_status s = rtc_get_state(c, saved.data());
  if (s != RTC_OK) return s;
  uint64_t *const tr0 = c->d_trace;
  const int32_t trf0 = c->trace_frames, trg0 = c->trace_groups;
  const std::vector<int32_t> split0 = c->split_h;
  const int32_t splitG0 = c->split_G;
  uint64_t *d_tr = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&d_tr, sizeof(uint64_t) * (size_t)n_frames * G * rtck::kTraceStages);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  auto cleanup = [&]() {
    c->d_trace = tr0;
    c->trace_frames = trf0;
    c->trace_groups = trg0;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (d_tr) (void)hipFree(d_tr);
  };
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(c, e, "rtc_balance_rows: allocation");
  }
  // one timed batch (after an untimed warm-up) in the current split; false on any failure
  auto timed = [&](float *us) -> bool {
    const int32_t warm = n_frames / 4 + 1;
    bool ok = rtc_frame_batch(c, std::min(warm, n_frames), d_pixels, frame_stride, d_cmd, nullptr, nullptr, nullptr,
                              nullptr, st) == RTC_OK;
    ok = ok && hipEventRecord(e0, st) == hipSuccess;
    ok = ok && rtc_frame_batch(c, n_frames, d_pixels, frame_stride, d_cmd, nullptr, nullptr, nullptr, nullptr,
                               st) == RTC_OK;
    ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float ms = 0.0f;
    ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    uint32_t aborted = 0;
    ok = ok && hipMemcpy(&aborted, c->d_sync + rtck::sync_layout::kSticky, sizeof(aborted), hipMemcpyDeviceToHost) ==
                   hipSuccess;
    ok = ok && aborted == 0;
    if (ok) *us = ms * 1000.0f / (float)n_frames;
    return ok;
  };
  // 1. the equal split: one traced batch, then one timed batch without the trace
  float t_eq = -1.0f, t_sp = -1.0f, t_tr = -1.0f;
  bool ok = rtc_set_row_split(c, 0, nullptr) == RTC_OK;
  c->d_trace = d_tr;
  c->trace_frames = n_frames;
  c->trace_groups = G;
  ok = ok && hipMemset(d_tr, 0, sizeof(uint64_t) * (size_t)n_frames * G * rtck::kTraceStages) == hipSuccess;
  ok = ok && timed(&t_tr);
  std::vector<uint64_t> tr((size_t)n_frames * G * rtck::kTraceStages);
  ok = ok && hipMemcpy(tr.data(), d_tr, tr.size() * sizeof(uint64_t), hipMemcpyDeviceToHost) == hipSuccess;
  c->d_trace = nullptr;
  c->trace_frames = 0;
  c->trace_groups = 0;
  ok = ok && timed(&t_eq);
  // 2. rows per second of every workgroup: median partial-sum time over the
  // last three quarters of the frames
  std::vector<double> rate((size_t)G, 0.0);
  bool traced = false;                             // no stamp at all: the batch did not run persistent
  for (const uint64_t v : tr) traced = traced || v != 0;
  for (int b = 0; ok && traced && b < G; ++b) {
    std::vector<double> d;
    for (int32_t f = n_frames / 4; f < n_frames; ++f) {
      const uint64_t *t = tr.data() + ((size_t)f * G + b) * rtck::kTraceStages;
      if (t[4] > t[3] && t[3] != 0) d.push_back((double)(t[4] - t[3]));
    }
    if (d.empty()) {
      ok = false;
      break;
    }
    std::nth_element(d.begin(), d.begin() + d.size() / 2, d.end());
    const int64_t r0 = (int64_t)b * c->n_act / G, r1 = (int64_t)(b + 1) * c->n_act / G;
    rate[(size_t)b] = (double)(r1 - r0) / d[d.size() / 2];
  }
  // 3. the proportional split, timed; keep the faster
  if (ok && traced) {
    const std::vector<int32_t> start = proportional_split(rate, c->n_act, 512);
    ok = rtc_set_row_split(c, G, start.data()) == RTC_OK && timed(&t_sp);
    if (ok && !(t_sp < t_eq)) ok = rtc_set_row_split(c, 0, nullptr) == RTC_OK;
  }
  if (!ok) {                                       // leave the caller's split
    (void)hipGetLastError();
    (void)hipDeviceSynchronize();
    (void)hipMemset(c->d_sync + rtck::sync_layout::kSticky, 0, sizeof(uint32_t));
    (void)rtc_set_row_split(c, splitG0, splitG0 > 0 ? split0.data() : nullptr);
  }
  if (ok && !traced) {
    ok = false;
    cleanup();
    (void)rtc_set_state(c, saved.data());
    (void)rtc_set_row_split(c, splitG0, splitG0 > 0 ? split0.data() : nullptr);
    return fail(c, RTC_E_STATE, "rtc_balance_rows: the persistent launch does not support this shape");
  }
  cleanup();
  s = rtc_set_state(c, saved.data());
  if (!ok) return fail(c, RTC_E_DEVICE, "rtc_balance_rows: a measurement batch failed");
  if (us_equal) *us_equal = t_eq;
  if (us_split) *us_split = t_sp;
  return s;
}

rtc_status rtc_calibrate_centroid(rtc_ctx *c, const uint16_t *d_pixels, float *d_slopes, int32_t *d_counts,
                                  void *hip_stream) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_calibrate_centroid: NULL context");
  if (!c->calib_loaded) return fail(c, RTC_E_STATE, "rtc_calibrate_centroid: load the calibration first");
  if (!d_pixels || !d_slopes) return fail(c, RTC_E_ARG, "rtc_calibrate_centroid: NULL pixels or slopes");
  DeviceScope ds(c->device);
  if (ds.status != hipSuccess) return hip_fail(c, ds.status, "rtc_calibrate_centroid: hipSetDevice");
  rtck::CalibArgs ca = calib_args(c, d_pixels);
  ca.s_int = d_slopes;     // the caller's vector is the only output
  ca.s_user = nullptr;
  ca.counts = d_counts;
  ca.ts_start = nullptr;
  hipError_t e = rtck::launch_calib_cog(ca, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(c, e, "rtc_calibrate_centroid: launch");
  return RTC_OK;
}

rtc_status rtc_reconstruct_integrate(rtc_ctx *c, const float *d_slopes, float *d_cmd, float *d_recon,
                                     void *hip_stream) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_reconstruct_integrate: NULL context");
  if (!c->cmat_loaded) return fail(c, RTC_E_STATE, "rtc_reconstruct_integrate: load the control matrix first");
  if (c->state_invalid) return fail(c, RTC_E_STATE, "rtc_reconstruct_integrate: " STATE_INVALID_MSG);
  if (!d_slopes || !d_cmd) return fail(c, RTC_E_ARG, "rtc_reconstruct_integrate: NULL slopes or cmd");
  DeviceScope ds(c->device);
  if (ds.status != hipSuccess) return hip_fail(c, ds.status, "rtc_reconstruct_integrate: hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const float *s = d_slopes;
  const int epc = rtck::format_elems_per_chunk(c->fmt);
  if ((c->n_slopes % epc) != 0 || (reinterpret_cast<uintptr_t>(d_slopes) & 15) != 0) {
    // the kernel reads 16-byte vectors of a zero-padded vector: stage a copy
    hipError_t e = hipMemcpyAsync(c->d_s, d_slopes, c->n_slopes * sizeof(float), hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(c, e, "rtc_reconstruct_integrate: slope copy");
    s = c->d_s;
  }
  rtck::MvmArgs ma{};
  ma.n_act = c->n_act;
  ma.n_s4 = c->n_s4;
  ma.s = s;
  ma.k_split = c->tuning.k_split;
  ma.rows_per_wave = c->tuning.rows_per_wave;
  ma.unroll = c->tuning.unroll;
  ma.part = c->d_part;
  ma.state = c->d_state;
  ma.cmd = d_cmd;
  ma.recon = d_recon;
  ma.gain = c->cfg.gain;
  ma.leak = c->cfg.leak;
  ma.cmd_min = c->cfg.cmd_min;
  ma.cmd_max = c->cfg.cmd_max;
  ma.sync = c->d_sync;
  ma.ts_end = nullptr;
  hipError_t e = launch_reconstruction(c, ma, st);
  if (e != hipSuccess) return hip_fail(c, e, "rtc_reconstruct_integrate: launch");
  return RTC_OK;
}

rtc_status rtc_set_mvm_tuning(rtc_ctx *c, const rtc_mvm_tuning *t) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_set_mvm_tuning: NULL context");
  if (!t) return fail(c, RTC_E_ARG, "rtc_set_mvm_tuning: NULL tuning");
  if (t->kernel == RTC_MVM_ROWBLOCK) {
    if (t->waves != 8 && t->waves != 16)
      return fail(c, RTC_E_ARG, "rtc_set_mvm_tuning: waves must be 8 or 16");
    if (t->rows_per_wave < 1 || t->rows_per_wave > 8)
      return fail(c, RTC_E_ARG, "rtc_set_mvm_tuning: rows_per_batch must be in 1..8");
    if (t->blocks < 0 || t->blocks > (1 << 20))
      return fail(c, RTC_E_ARG, "rtc_set_mvm_tuning: blocks must be in 0..2^20");
  } else if (t->kernel == RTC_MVM_STREAMED) {
    if (c->fmt != RTC_CM_F32)
      return fail(c, RTC_E_UNSUPPORTED, "rtc_set_mvm_tuning: the streamed kernel reads float32 matrices only");
    if (t->k_split < 1 || t->k_split > rtck::kMaxKSplit)
      return fail(c, RTC_E_ARG, "rtc_set_mvm_tuning: k_split must be in 1..64");
    if (!rtck::mvm_variant_supported(t->rows_per_wave, t->unroll))
      return fail(c, RTC_E_ARG, "rtc_set_mvm_tuning: unsupported rows_per_wave/unroll pair");
  } else {
    return fail(c, RTC_E_ARG, "rtc_set_mvm_tuning: unknown kernel");
  }
  c->tuning = *t;
  return RTC_OK;
}

rtc_status rtc_get_mvm_tuning(const rtc_ctx *c, rtc_mvm_tuning *t) {
  if (!c || !t) return fail(nullptr, RTC_E_ARG, "rtc_get_mvm_tuning: NULL argument");
  *t = c->tuning;
  return RTC_OK;
}

rtc_status rtc_set_frame_mode(rtc_ctx *c, int32_t mode, int32_t spin_limit) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_set_frame_mode: NULL context");
  if (mode != RTC_FRAMES_PER_LAUNCH && mode != RTC_FRAMES_PERSISTENT && mode != RTC_FRAMES_HORIZONTAL)
    return fail(c, RTC_E_ARG, "rtc_set_frame_mode: unknown mode");
  if (spin_limit < 0) return fail(c, RTC_E_ARG, "rtc_set_frame_mode: spin_limit must be >= 0");
  if (mode == RTC_FRAMES_HORIZONTAL) {
    int32_t nch, nrt, nq;
    std::string why;
    if (!horiz_shape(c, &nch, &nrt, &nq, &why)) return fail(c, RTC_E_UNSUPPORTED, "rtc_set_frame_mode: " + why);
    DeviceScope ds(c->device);
    if (ds.status != hipSuccess) return hip_fail(c, ds.status, "rtc_set_frame_mode: hipSetDevice");
    if (c->h_gen != c->cmat_gen) {
      const rtc_status st = horiz_prepare(c, "rtc_set_frame_mode");
      if (st != RTC_OK) return st;
    }
  }
  c->frame_mode = mode;
  c->spin_limit = spin_limit > 0 ? spin_limit : (1 << 22);
  return RTC_OK;
}

rtc_status rtc_get_frame_mode(const rtc_ctx *c, int32_t *mode) {
  if (!c || !mode) return fail(nullptr, RTC_E_ARG, "rtc_get_frame_mode: NULL argument");
  *mode = c->frame_mode;
  return RTC_OK;
}

rtc_status rtc_set_trace(rtc_ctx *c, uint64_t *d_trace, int32_t max_frames, int32_t n_groups) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_set_trace: NULL context");
  if (max_frames < 0 || (max_frames > 0 && !d_trace))
    return fail(c, RTC_E_ARG, "rtc_set_trace: need a buffer for max_frames > 0");
  if (max_frames > 0 && (n_groups < 1 || n_groups > 4096))
    return fail(c, RTC_E_ARG, "rtc_set_trace: n_groups must be in [1, 4096]");
  c->d_trace = max_frames > 0 ? d_trace : nullptr;
  c->trace_frames = max_frames;
  c->trace_groups = max_frames > 0 ? n_groups : 0;
  return RTC_OK;
}

rtc_status rtc_sync_check(rtc_ctx *c) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_sync_check: NULL context");
  DeviceScope ds(c->device);
  hipError_t e = ds.status;
  uint32_t flag = 0;
  if (e == hipSuccess) e = hipDeviceSynchronize();
  uint32_t *sticky = c->d_sync + rtck::sync_layout::kSticky;
  if (e == hipSuccess) e = hipMemcpy(&flag, sticky, sizeof(flag), hipMemcpyDeviceToHost);
  if (e == hipSuccess && flag) e = hipMemset(sticky, 0, sizeof(uint32_t));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(c, e, "rtc_sync_check");
  if (flag) {
    c->state_invalid = true;
    return fail(c, RTC_E_DEVICE, "rtc_sync_check: a persistent or pixel-stream batch gave up at a bounded "
                                 "wait; the frame that waited and later ones were not processed and the "
                                 "integrator state is undefined until rtc_reset or rtc_set_state");
  }
  return RTC_OK;
}

rtc_status rtc_reset(rtc_ctx *c) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_reset: NULL context");
  DeviceScope ds(c->device);
  hipError_t e = ds.status;
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemset(c->d_state, 0, c->n_act * sizeof(float));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) c->state_invalid = false;
  return e == hipSuccess ? RTC_OK : hip_fail(c, e, "rtc_reset");
}

rtc_status rtc_get_state(rtc_ctx *c, float *h_cmd) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_get_state: NULL context");
  if (!h_cmd) return fail(c, RTC_E_ARG, "rtc_get_state: NULL output");
  DeviceScope ds(c->device);
  hipError_t e = ds.status;
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(h_cmd, c->d_state, c->n_act * sizeof(float), hipMemcpyDeviceToHost);
  return e == hipSuccess ? RTC_OK : hip_fail(c, e, "rtc_get_state");
}

rtc_status rtc_set_state(rtc_ctx *c, const float *h_cmd) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_set_state: NULL context");
  if (!h_cmd) return fail(c, RTC_E_ARG, "rtc_set_state: NULL input");
  for (int32_t i = 0; i < c->n_act; ++i)
    if (!std::isfinite(h_cmd[i])) return fail(c, RTC_E_NONFINITE, "rtc_set_state: non-finite value");
  DeviceScope ds(c->device);
  hipError_t e = ds.status;
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(c->d_state, h_cmd, c->n_act * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) c->state_invalid = false;
  return e == hipSuccess ? RTC_OK : hip_fail(c, e, "rtc_set_state");
}

rtc_status rtc_wall_clock_khz(rtc_ctx *c, int64_t *khz) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_wall_clock_khz: NULL context");
  if (!khz) return fail(c, RTC_E_ARG, "rtc_wall_clock_khz: NULL output");
  *khz = c->wall_khz;
  return RTC_OK;
}

rtc_status rtc_probe_copy(rtc_ctx *c, const void *d_src, void *d_dst, int64_t n_bytes, void *hip_stream) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_probe_copy: NULL context");
  if (!d_src || !d_dst || n_bytes < 0 || (n_bytes & 15))
    return fail(c, RTC_E_ARG, "rtc_probe_copy: NULL pointer or size not a multiple of 16");
  DeviceScope ds(c->device);
  if (ds.status != hipSuccess) return hip_fail(c, ds.status, "rtc_probe_copy: hipSetDevice");
  hipError_t e = rtck::launch_probe_copy(d_src, d_dst, n_bytes, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? RTC_OK : hip_fail(c, e, "rtc_probe_copy: launch");
}

rtc_status rtc_probe_read(rtc_ctx *c, const void *d_src, int64_t n_bytes, float *d_out, void *hip_stream) {
  if (!c) return fail(nullptr, RTC_E_ARG, "rtc_probe_read: NULL context");
  if (!d_src || !d_out || n_bytes < 0 || (n_bytes & 15))
    return fail(c, RTC_E_ARG, "rtc_probe_read: NULL pointer or size not a multiple of 16");
  DeviceScope ds(c->device);
  if (ds.status != hipSuccess) return hip_fail(c, ds.status, "rtc_probe_read: hipSetDevice");
  hipError_t e = rtck::launch_probe_read(d_src, n_bytes, d_out, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? RTC_OK : hip_fail(c, e, "rtc_probe_read: launch");
}

void rtc_destroy(rtc_ctx *c) {
  if (!c) return;
  DeviceScope ds(c->device);
  if (ds.status == hipSuccess) (void)hipDeviceSynchronize();
  dfree(c->d_tiles);
  dfree(c->d_calib);
  dfree(c->d_ref);
  dfree(c->d_R);
  dfree(c->d_scales);
  dfree(c->d_s);
  dfree(c->d_state);
  dfree(c->d_part);
  dfree(c->d_sbuf);
  dfree(c->d_sync);
  dfree(c->d_row_start);
  dfree(c->d_packed);
  dfree(c->d_ppart);
  dfree(c->d_ring);
  dfree(c->d_psync);
  dfree(c->d_first);
  dfree(c->d_need);
  dfree(c->d_hm);
  dfree(c->d_xbuf);
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  if (c->h_trig) (void)hipHostFree(c->h_trig);
  delete c;
}

}  // extern "C"

namespace rtcx {

rtc_status enqueue_frame_with(rtc_ctx *c, const uint16_t *pix, float *cmd, float *slopes, float *recon,
                              int32_t *counts, uint64_t *ts, hipStream_t st, const char *who, SlopeStep step,
                              void *arg) {
  return enqueue_frame(c, ctx_scratch(c), pix, cmd, slopes, recon, counts, ts, st, who, step, arg);
}

rtc_status enqueue_pred_frames(rtc_ctx *c, const rtcm::PredStepArgs &q, int32_t seen, int32_t n_frames,
                               const uint16_t *d_pixels, int64_t frame_stride, float *d_cmd, float *d_slopes,
                               uint64_t *d_ts, hipStream_t st, const char *who, bool *ran) {
  *ran = false;
  if (c->frame_mode != RTC_FRAMES_PERSISTENT || n_frames <= 0) return RTC_OK;
  rtck::PersistArgs p = persist_args(c, n_frames, d_pixels, frame_stride, d_cmd, d_slopes, nullptr, nullptr, d_ts);
  p.trace = nullptr;                                // the stage trace covers plain frames only
  p.pred = q;
  p.pred_seen = seen;
  p.sbuf_pred = c->d_sbuf + 2 * xchg_len_of(c->n_slopes);
  const int blocks = c->tuning.blocks > 0 ? c->tuning.blocks : c->n_cu;
  const int G = rtck::frames_grid(blocks, c->n_act);
  p.calib_span = calib_span(c, G);
  if (c->split_G > 0 && c->split_G == G) {
    p.row_start = c->d_row_start;
    p.row_max = c->split_max;
  }
  const hipError_t e = rtck::launch_frames(p, blocks, c->tuning.rows_per_wave, st);
  if (e == hipErrorInvalidValue || e == hipErrorCooperativeLaunchTooLarge) {
    (void)hipGetLastError();                        // shape not built: the caller runs per-launch frames
    return RTC_OK;
  }
  if (e != hipSuccess) return hip_fail(c, e, who);
  *ran = true;
  return RTC_OK;
}

}  // namespace rtcx
