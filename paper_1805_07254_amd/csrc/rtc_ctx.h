// Internal: the context object behind rtc_ctx* and the host helpers shared by
// the C-ABI source files.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/rtc.h"
#include "rtc_kernels.h"

// One wavefront sensor of a context.
struct WfsInfo {
  int32_t n_sub_x = 0, n_sub_y = 0, n_pix = 0, H = 0, W = 0;
  int64_t frame_off = 0;   // first element of its frame in the frame set
  int32_t tile_base = 0;   // its first subaperture
  int32_t n_tiles = 0;
};

struct rtc_ctx {
  rtc_config cfg{};        // abi_version, n_act, thr_mode, cm_dtype, gain, leak, clamp, device
  int device = 0;
  int32_t n_valid = 0, n_slopes = 0, n_s4 = 0, n_act = 0;
  std::vector<WfsInfo> wfs;
  int64_t frame_elems = 0;  // elements of one frame set
  int32_t max_n = 0;        // largest pixels per side
  int32_t pairs = 0;        // every tile row starts on an even element and has even width
  int64_t calib_len = 0;    // float2 elements of the per-tile calibration blocks
  int64_t ldr = 0;        // float32 row length of the matrix (elements)
  int64_t s_len = 0;      // slope / reference buffer length (elements)
  int32_t fmt = 0;        // rtc_cm_dtype of the stored matrix
  int64_t ldq = 0;        // stored row length (elements)
  int32_t n_chunks = 0;   // 16-byte chunks per stored row
  std::vector<rtck::TileDesc> tiles_h;
  std::string err;
  rtc_mvm_tuning tuning{RTC_MVM_ROWBLOCK, 1, 2, 4, 0, 8};
  int32_t n_cu = 0;
  int64_t wall_khz = 0;

  rtck::TileDesc *d_tiles = nullptr;
  float2 *d_calib = nullptr;
  float *d_ref = nullptr;
  void *d_R = nullptr;
  float *d_scales = nullptr;
  float *d_s = nullptr;
  float *d_state = nullptr;
  float *d_part = nullptr;
  float *d_sbuf = nullptr;   // [4][s_len]: slope vectors of consecutive frames (persistent batches), then
                             // the feed-forward slopes of consecutive predictive frames
  uint32_t *d_sync = nullptr;  // rtck::sync_layout words: stamp counter, abort flags, persistent barrier
  uint32_t *d_scratch = nullptr;  // this device's static scratch array (rtc_frame_batch_noalloc); not owned
  uint32_t *h_trig = nullptr;      // coherent host words of paced batches: [0] release, [32] done
  uint32_t trig_base = 0;          // frames released by earlier paced batches (mod 2^32)
  int32_t frame_mode = RTC_FRAMES_PER_LAUNCH;
  int32_t spin_limit = 1 << 22;
  uint64_t *d_trace = nullptr;  // caller-owned [trace_frames][trace_groups][8] stage stamps
  int32_t trace_frames = 0;
  int32_t trace_groups = 0;
  hipGraphExec_t graph = nullptr;  // recorded frame batch (rtc_graph_capture)
  int32_t *d_row_start = nullptr;  // [kMaxGroups + 1] measured row split of persistent batches
  int32_t split_G = 0;             // grid the split is for (0 = equal split)
  int32_t split_max = 0;           // most rows of one workgroup in the split
  std::vector<int32_t> split_h;    // host copy of the split (split_G + 1 entries)
  int32_t dark_fast = 1;           // every loaded dark is 0 or of magnitude in [2^-13, 2^24)
  // horizontal frames (RTC_FRAMES_HORIZONTAL): the matrix in the per-workgroup
  // layout and the partial-vector messages
  uint4 *d_hm = nullptr;
  int64_t hm_chunks = 0;
  float *d_xbuf = nullptr;
  uint64_t h_gen = 0;              // cmat_gen the layout was built from (0 = none)
  int32_t h_nch = 0, h_nrt = 0, h_nq = 0;
  bool calib_loaded = false;
  bool state_invalid = false;      // a reported failed batch left the integrator state undefined
  bool cmat_loaded = false;
  uint64_t cmat_gen = 0;           // bumped by every rtc_load_cmat

  // pixel-stream processing (rtc_pipe_setup)
  uint64_t pipe_gen = 0;           // cmat_gen the packed columns were made from; 0 = not set up
  rtc_pipe_config pipe_cfg{};
  int32_t pipe_workers = 0, pipe_lds_cols = 0, pipe_max_nb = 0, pipe_H = 0, pipe_W = 0;
  int32_t pipe_n_tail = 0, pipe_own_max = 0, pipe_n_own = 0;
  int64_t pipe_ldp = 0, pipe_ring_stride = 0;
  size_t pipe_lds = 0;
  void *d_packed = nullptr;        // [2 n_valid][ldp] codes
  float *d_ppart = nullptr;        // [2][workers][ldp]
  uint16_t *d_ring = nullptr;      // [2][ring_stride]
  uint32_t *d_psync = nullptr;     // rtck::pipe_layout words
  int32_t *d_first = nullptr;      // [workers + 1]
  int32_t *d_need = nullptr;       // [n_valid]
};

// Frame calls refuse to run on a state that a failed persistent or pixel-stream
// batch left undefined.
#define STATE_INVALID_MSG "a failed batch left the integrator state undefined; call rtc_reset or rtc_set_state"

namespace rtcx {

inline thread_local std::string g_init_err = "no error";

inline rtc_status fail(rtc_ctx *c, rtc_status s, const std::string &msg) {
  if (c) c->err = msg; else g_init_err = msg;
  return s;
}

inline rtc_status hip_fail(rtc_ctx *c, hipError_t e, const char *what) {
  std::string m = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  return fail(c, e == hipErrorOutOfMemory ? RTC_E_NOMEM : RTC_E_DEVICE, m);
}

// Makes the context's device current for the scope and restores the caller's.
struct DeviceScope {
  int prev = -1;
  hipError_t status = hipSuccess;
  explicit DeviceScope(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    status = hipSetDevice(dev);
  }
  ~DeviceScope() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

template <typename T>
inline void dfree(T *&p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// A step between a frame's slopes and its reconstruction: given the slopes s
// and the commands c_prev of the previous frame (the integrator state), it
// enqueues its work on st and returns in *s_use the slope vector the
// reconstruction multiplies (zero-padded like the library's own).
using SlopeStep = hipError_t (*)(void *arg, const float *s, const float *c_prev, const float **s_use,
                                 hipStream_t st);

// One per-launch frame (calibration, step, reconstruction and integrator) on
// st, as a frame of rtc_frame_batch in the per-launch mode; ts (nullable) gets
// its start and end stamps.
rtc_status enqueue_frame_with(rtc_ctx *c, const uint16_t *pix, float *cmd, float *slopes, float *recon,
                              int32_t *counts, uint64_t *ts, hipStream_t st, const char *who, SlopeStep step,
                              void *arg);

// Predictive frames in one persistent launch when the context is in the
// persistent mode and the built kernels cover its shape (*ran = true); the
// step's arguments q (vectors and per-frame flags are set by the kernel), its
// ring slot q.pos and the frames it has seen (seen) before the batch.
// *ran = false: nothing was enqueued, the caller runs per-launch frames.
rtc_status enqueue_pred_frames(rtc_ctx *c, const rtcm::PredStepArgs &q, int32_t seen, int32_t n_frames,
                               const uint16_t *d_pixels, int64_t frame_stride, float *d_cmd, float *d_slopes,
                               uint64_t *d_ts, hipStream_t st, const char *who, bool *ran);

}  // namespace rtcx
