// Internal interface between the C-ABI host code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pred_step.h"

namespace rtck {

// One active subaperture (32 bytes): where its pixels and calibration are,
// where its slopes go, and its sensor's geometry and threshold.
struct TileDesc {
  int32_t off;             // element offset of its top-left pixel in the frame set
  int32_t calib_off;       // float2 offset of its [n][n] (dark, flat) block
  int32_t sx, sy;          // positions of its x and y slopes in the slope vector
  int32_t pitch;           // row length of its sensor's frame (elements)
  int32_t n;               // pixels per side, 1..32
  float thr;               // its sensor's threshold
  int32_t reserved;
};

// Steps (a)-(b): calibration + centre of gravity of every active subaperture.
struct CalibArgs {
  const uint16_t *pix;     // frame set
  const TileDesc *tiles;   // [n_valid]
  const float2 *calib;     // per-tile (dark, flat) blocks
  int32_t n_valid;
  int32_t max_n;           // largest tile side (lanes per tile)
  int32_t pairs;           // every tile row starts on an even element and has even width
  int32_t mode;            // threshold: 0 = none, 1 = subtract, 2 = zero
  int32_t dark_fast;       // 1: every dark is 0 or of magnitude in [2^-13, 2^24) (raw - dark exact in float64)
  const float *ref;        // [n_slopes] reference slopes (by slope position)
  float *s_int;            // [>= n_slopes] library slope buffer
  float *s_user;           // nullable copy
  int32_t *counts;         // nullable [n_valid]
  uint64_t *ts_start;      // nullable: written by block 0 on entry
  int32_t xchg_epc;        // persistent batches: elements per chunk of the slope exchange layout
};
hipError_t launch_calib_cog(const CalibArgs &a, hipStream_t st);

// Steps (c)-(d): a = R s, then c = clamp(leak c + gain a).
struct MvmArgs {
  const float *R;          // float32 [n_act][ldr], ldr % 4 == 0 (streamed kernel)
  int64_t ldr;
  const void *Rq;          // [n_act] rows of ldq_bytes: codes of the storage format (row-block kernel)
  int64_t ldq_bytes;       // row pitch, multiple of 16
  const float *scales;     // [n_act] per-row scales, nullptr for float32 storage
  int32_t fmt;             // 0 float32, 1 binary16, 2 bfloat16, 3 FP8 E4M3 (OCP)
  int32_t n_chunks;        // 16-byte code chunks per row covering the slope vector
  int32_t n_act;
  int32_t n_s4;            // slope vector length / 4 (zero-padded)
  const float *s;          // slope vector, zero-padded to a multiple of 16 floats, 16-byte aligned
  int32_t k_split;         // partitions of the slope dimension (1 = fused epilogue)
  int32_t rows_per_wave;   // 1, 2 or 4 actuator rows per wavefront
  int32_t unroll;          // 2, 4 or 8 16-byte loads per row and lane in flight
  float *part;             // [k_split][n_act] partial sums (k_split > 1)
  float *state;            // [n_act] integrator state (read and updated)
  float *cmd;              // [n_act] commands out
  float *recon;            // nullable [n_act] a = R s
  float gain, leak, cmd_min, cmd_max;
  uint32_t *sync;          // completion counter (0 between launches)
  uint64_t *ts_end;        // nullable: written after the last workgroup's results
};
// Returns the number of slope partitions actually used (<= k_split) in *used.
hipError_t launch_mvm_integrate(const MvmArgs &a, int32_t *used, hipStream_t st);

bool mvm_variant_supported(int rows_per_wave, int unroll);

// A wavefront's slice of the 16-byte chunks of a row: whole groups of 64
// chunks (one per lane), so slices start on group boundaries.
__host__ __device__ inline int slice_chunks(int n_chunks, int waves) {
  return ((n_chunks + waves - 1) / waves + 63) / 64 * 64;
}

// Row-block reconstruction + integrator (no slope split): `blocks` workgroups of
// `waves` (8 or 16) wavefronts, `rows_per_batch` rows streamed per batch.
// Fails with hipErrorInvalidValue when a wavefront's slope slice would need
// more than mvm_block_max_kpl(fmt) 16-byte vectors per lane (8 wavefronts) or
// more than 8 (16 wavefronts).
hipError_t launch_mvm_block(const MvmArgs &a, int blocks, int waves, int rows_per_batch, hipStream_t st);
int mvm_block_max_kpl(int fmt);
// Row-block reconstruction over slope panels (8 wavefronts, any slope-vector
// length): used when 8 wavefronts' slices would exceed mvm_block_max_kpl(fmt)
// vectors per lane, with the slicing of the persistent kernel's panels.
hipError_t launch_mvm_panel(const MvmArgs &a, int blocks, hipStream_t st);
// Elements per 16-byte chunk of a storage format (4, 8, 8, 16).
int format_elems_per_chunk(int fmt);

// Persistent frames (steps (a)-(d) for n_frames frames in one cooperative launch).
struct PersistArgs {
  CalibArgs cal;           // pix = frame 0; s_user / counts = per-frame output bases (nullable)
  int64_t frame_stride;    // elements between frames
  int32_t n_frames;
  int32_t vec;             // 4-byte pixel pairs usable for every frame
  float *sbuf;             // [2][s_len] slope vectors of consecutive frames in the exchange layout, zero-padded
  int32_t s_len;           // >= round_up(chunks, 64) * 16 floats
  MvmArgs mvm;             // cmd / recon = per-frame output bases [n_frames][n_act]
  uint32_t *bar;           // sync words from sync_layout::kBarBase on (counters and mailboxes zeroed per launch)
  uint32_t *abort_flag;    // raised when a bounded wait expires (zeroed per launch)
  uint32_t *sticky;        // raised with abort_flag; cleared only by the host
  int32_t spin_limit;      // spins (about 30-60 ns each) before a wait gives up
  uint64_t *ts;            // nullable [n_frames][2]
  uint64_t *trace;         // nullable [trace_frames][trace_groups][kTraceStages] stage stamps
  int32_t trace_frames;
  int32_t trace_groups;
  int32_t calib_span;      // largest float2 count of one workgroup's (dark, flat) blocks for the
                           // grid of frames_grid(); 0 = not known (they are then read from memory)
  const int32_t *row_start;  // nullable [G + 1]: workgroup b owns rows [row_start[b], row_start[b+1])
  int32_t row_max;           // largest row_start[b+1] - row_start[b] (with row_start)
  // external frame trigger (nullable): frame f starts once *trig_release
  // reaches trig_base + f + 1 (coherent host memory, polled by workgroup 0 and
  // relayed to the others' mailbox lines); its commands are then stored at
  // system scope and the last workgroup to finish it writes trig_base + f + 1
  // to *trig_done
  const uint32_t *trig_release;
  uint32_t *trig_done;
  uint32_t trig_base;
  // predictive frames (pred.n_modes > 0): the learned predictor's step runs
  // between the slope exchange and the products, in four phases with a grid
  // barrier after each; the kernel sets its vectors (s, c, s_out) and the
  // per-frame push / full / pos, starting from ring slot pred.pos with
  // pred_seen frames seen (at most the history) before the launch.  Rows of
  // W1 and W2 must start 8-byte aligned with n_in and n_hid multiples of 4.
  rtcm::PredStepArgs pred;
  int32_t pred_seen;
  float *sbuf_pred;        // [2][s_len] feed-forward slopes in the exchange layout, zero-padded
};
constexpr int kTraceStages = 8;
// Zeroes the barrier counters, the mailboxes of G workgroups and the abort flag
// before a persistent launch (a kernel, so that it can be recorded in a graph).
hipError_t launch_persist_reset(uint32_t *bar, uint32_t *abort_flag, int G, hipStream_t st);

// Synchronisation words of a context, in uint32 units.  Arrival counters sit
// 4 KiB apart so that arrivals and polls at different counters do not queue at
// one memory channel, and a barrier is released by writing the frame number
// into one 64-byte mailbox per workgroup, so that every workgroup polls a line
// of its own.  Offsets from kMailbox on are relative to kBarBase.
namespace sync_layout {
constexpr int kStampCounter = 0, kAbort = 1, kSticky = 2;
constexpr int kBarBase = 1024;
constexpr int kStride = 1024;
constexpr int kGroups = 16;                       // group g arrival counter at kStride * g
constexpr int kTop = kGroups * kStride;           // arrivals of whole groups
constexpr int kDone = (kGroups + 1) * kStride;    // workgroups done with a batch (end stamp)
constexpr int kTrigDone = kDone + 16;             // workgroups done with triggered frames
constexpr int kMailbox = (kGroups + 2) * kStride; // + 16 * workgroup: [0] barrier epoch, [4] trigger relay
constexpr int kMaxGroups = 1024;
constexpr int kEnds = kMailbox + 16 * kMaxGroups; // uint64 [3][kMaxGroups] per-workgroup frame end stamps
constexpr int kEndSlots = 3;                      // rows of end stamps (frame f in row f mod 3)
constexpr int kWords = kBarBase + kEnds + 2 * kEndSlots * kMaxGroups;
}  // namespace sync_layout
// Fails with hipErrorInvalidValue when the shape is unsupported (slab rows
// beyond one per thread, LDS, register slices) and with the runtime's error
// when the grid cannot be co-resident.
hipError_t launch_frames(const PersistArgs &p, int blocks, int rows_per_batch, hipStream_t st);
// Workgroups of a persistent launch asked for `blocks` workgroups (workgroup b
// owns subapertures [b n_valid / G, (b + 1) n_valid / G)).
int frames_grid(int blocks, int n_act);

// Persistent frames in the horizontal split (the paper's processing strategy,
// Section 2.2 and Figure 5): kHoriz workgroups, one per compute unit, of
// kHoriz threads.  Workgroup b calibrates subapertures [b n_valid / G,
// (b+1) n_valid / G) and multiplies their slopes into its own columns of the
// control matrix (every actuator row), which stay on chip for the whole batch:
// a partial actuator vector.  Thread t of every workgroup computes the rows of
// owner t, [rb(t), rb(t+1)) with rb(o) = o q + min(o, rem), q = n_act / G,
// rem = n_act % G, and stores them as producer b's message to owner t.  After
// the frame barrier, owner b adds the G messages of its rows in a fixed order
// (the tree vector addition of Section 2.3.5 as a reduce-scatter) and applies
// the integrator.
constexpr int kHoriz = 256;          // workgroups of a launch = threads of a workgroup
constexpr int kHorizMsg = 32;        // floats per message (rows of an owner, zero-padded)

struct HorizArgs {
  PersistArgs p;           // calibration, frames, outputs, integrator and sync words (row split unused)
  const uint4 *hm;         // horizontal layout [G][nrt][nq][kHoriz] 16-byte chunks (horiz_layout)
  float *xbuf;             // [2][G owners][G producers][kHorizMsg] messages, zero-initialised
  int32_t nch;             // subapertures per workgroup (columns: nch x slopes, then nch y slopes)
  int32_t nrt;             // rows of the largest owner (row slots per thread)
};
// Chunks per row slot the horizontal kernel is built for (16-byte chunks of a
// workgroup's 2 nch columns), 0 when 2 nch is too wide for the format.
int horiz_chunks(int fmt, int nch);
// Most rows per owner the instantiated horizontal kernels of a format and
// chunk count hold (registers and LDS tail slots); 0 when none is built.
int horiz_max_rows(int fmt, int nq);
// Elements of the horizontal layout (uint4 chunks).
int64_t horiz_layout_chunks(int G, int nrt, int nq);
// Builds the horizontal layout from the stored row-major matrix Rq (rows of
// ldq_bytes, codes of format fmt): chunk (b, i, q, t) = codes of row
// rb(t) + i at the columns [q EPC, (q+1) EPC) of workgroup b.
hipError_t launch_horiz_layout(const void *Rq, int64_t ldq_bytes, int fmt, const TileDesc *tiles, int n_valid,
                               int n_act, int G, int nch, int nrt, int nq, uint4 *hm, hipStream_t st);
// Zeroes n floats (graph-safe: a kernel, not a memset).
hipError_t launch_fill_zero(float *p, int64_t n, hipStream_t st);
// Cooperative launch of the horizontal frames; hipErrorInvalidValue for
// shapes it does not cover.
hipError_t launch_horizontal(const HorizArgs &h, hipStream_t st);

// Pixel-stream frames: a camera workgroup lands the rows of each frame in a
// two-slot ring on a schedule (rows of frame f land uniformly over the readout
// time from f * frame period on) and publishes a landed-row counter; every
// other workgroup (a worker) owns a contiguous run of subapertures in arrival
// order and, as soon as their rows have landed, calibrates them, centroids
// them and multiplies their slopes into the matching columns of the control
// matrix (a partial actuator vector).  The first n_own workers also own
// actuator rows (owner b: [b n_act / n_own, (b+1) n_act / n_own)): each sums
// the P partial vectors of its rows in worker order and applies the
// integrator.
namespace pipe_layout {
constexpr int kStride = 1024;                     // 4 KiB between counters
constexpr int kRowCopies = 16;                    // landed-row counter copies, worker b polls copy b % 16
constexpr int kFlags = kRowCopies * kStride;      // + 16 * worker: frames whose partial vector is published
constexpr int kMaxWorkers = 1024;
constexpr int kOwnDone = kFlags + 16 * kMaxWorkers;   // workers done with a frame (all their rows integrated)
constexpr int kWords = kOwnDone + kStride;
constexpr int kMaxQuadsPerThread = 4;             // packed column length <= 4 * 4 * 512 codes
constexpr int kCamStamps = 4;                     // per frame: scheduled start, first rows, last rows, worst slip
}  // namespace pipe_layout

struct PipeArgs {
  const TileDesc *tiles;   // [n_valid] (one sensor: off is relative to the frame start)
  const float2 *calib;
  const float *ref;
  int32_t n_valid;
  int32_t max_n;
  int32_t mode;            // threshold: 0 = none, 1 = subtract, 2 = zero
  int32_t dark_fast;       // as CalibArgs::dark_fast
  int32_t fmt;             // storage format of the packed columns
  // camera
  const uint16_t *src;     // [n_frames] frames, src_stride elements apart, 4-byte aligned
  int64_t src_stride;
  uint16_t *ring;          // [2][ring_stride] landing slots
  int64_t ring_stride;     // elements, multiple of 128
  int64_t frame_elems;     // even
  int32_t H, W;            // image rows and row length (elements)
  int32_t rows_per_packet;
  int32_t n_frames;
  double t_frame, t_row;   // wall-clock ticks
  int64_t lead;            // ticks from the camera's start to frame 0
  int64_t wait_ticks;      // a wait gives up after this long
  // workers
  const int32_t *first;    // [P + 1] first subaperture of each worker
  const int32_t *need;     // [n_valid] image rows a subaperture needs
  const void *packed;      // [2 n_valid][ldp] codes: column 2k = x slope of subaperture k, 2k + 1 = y slope
  int64_t ldp;             // codes per packed column, multiple of 64
  int32_t lds_cols;        // trailing columns of a worker kept in LDS
  int32_t max_nb;          // most subapertures of a worker
  int32_t n_tail;          // subapertures [n_valid - n_tail, n_valid): every owner processes them for its own rows
  int32_t n_own;           // owners: workers [0, n_own) hold the actuator rows
  int32_t own_max;         // most actuator rows of an owner (<= 64)
  int32_t n_act;
  const float *scales;     // nullable [n_act]
  float *state;            // [n_act]
  float *cmd;              // [n_frames][n_act]
  float *recon;            // nullable [n_frames][n_act]
  float gain, leak, cmd_min, cmd_max;
  float *part;             // [2][P][ldp] partial actuator vectors
  float *s_user;           // nullable [n_frames][2 n_valid]
  int32_t *counts;         // nullable [n_frames][n_valid]
  uint32_t *sync;          // pipe_layout words (zeroed per launch)
  uint32_t *abort_flag;    // zeroed per launch
  uint32_t *sticky;
  uint64_t *cam_ts;        // nullable [n_frames][kCamStamps]
  uint64_t *wk_ts;         // nullable [n_frames][P][2]: partial published, rows integrated
};
// G = P + 1 workgroups of 512 threads; lds_bytes of dynamic LDS per workgroup.
hipError_t launch_pipe(const PipeArgs &p, int G, size_t lds_bytes, hipStream_t st);
// LDS bytes a worker needs besides its columns.
size_t pipe_lds_fixed(int max_nb, int n_tail, int own_max);
constexpr int kPipeMaxTail = 64;                   // tail subapertures (two slope columns per lane)
constexpr int kPipeStaticLds = 4096;               // static shared memory of the pipe kernel (upper bound)
// Bytes per code of a storage format (4, 2, 2, 1).
int format_code_bytes(int fmt);
// packed[(2k + h) ldp + r] = code of row r, slope column (h ? tiles[k].sy : tiles[k].sx); rows
// n_act..ldp-1 zero.
hipError_t launch_pack_columns(const void *Rq, int64_t ldq_bytes, int fmt, const TileDesc *tiles, int n_valid,
                               int n_act, void *packed, int64_t ldp, hipStream_t st);

// Roofline probes.
hipError_t launch_probe_copy(const void *src, void *dst, int64_t n_bytes, hipStream_t st);
hipError_t launch_probe_read(const void *src, int64_t n_bytes, float *out, hipStream_t st);

constexpr int kMaxKSplit = 64;
constexpr int kMaxChunk4 = 4096;   // slope floats staged in LDS per workgroup / 4 (64 KiB)

}  // namespace rtck
