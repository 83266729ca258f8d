/*
 * rtc.h -- C ABI of the MI355X (gfx950) adaptive-optics real-time-control hot path.
 *
 * One frame of a single-conjugate AO real-time controller, as the paper lays it
 * out (Jenkins, Basden & Myers 2018, "ELT-scale Adaptive Optics real-time
 * control with the Intel Xeon Phi Many Integrated Core Architecture",
 * Section 2.1 and the Figure 3 caption):
 *
 *   (a) pixel calibration of each active Shack-Hartmann subaperture:
 *       background (dark) subtraction, flat-field application, threshold;
 *   (b) centre-of-gravity centroids, written into the slope vector with all x
 *       gradients first and then all y gradients (subaperture i -> s_i and
 *       s_{n/2+i});
 *   (c) reconstruction: control matrix (actuators x slopes) times slope vector
 *       (Section 1.1.1; Figure 3 (c));
 *   (d) a gain applied to the reconstruction, here an integrator
 *       c_k = leak * c_{k-1} + gain * a_k, clamped, giving the DM commands.
 *
 * Every step runs in hand-written HIP kernels on the device given at init.
 *
 * Conventions
 *  - All scalars at the boundary are float32.  No HIP or torch types appear:
 *    streams are passed as `void *` (a hipStream_t, NULL = the null stream).
 *  - Host arrays passed to rtc_init / rtc_load_* are COPIED; the caller keeps
 *    ownership.  The library owns its device copies and may re-lay them out.
 *  - Frame inputs and outputs are caller-owned DEVICE pointers on the context's
 *    device.  Frame calls are asynchronous on the given stream; completion is
 *    observed through that stream.
 *  - Every call returns an rtc_status.  On any error nothing is modified
 *    (loads validate everything before touching device state).
 *    rtc_error_string() gives the last error text.
 *  - A context is not thread-safe: one host thread per context.  Several
 *    contexts may coexist.  Frame calls on one context must be issued in frame
 *    order; calls on different streams of the same context race.
 *
 * Threshold decision: a pixel is "above" when the exact real number
 * (raw - dark) * flat - T is > 0 (a tie counts as below), for every finite
 * float32 dark and flat.  When every dark is 0 or of magnitude in [2^-13, 2^24)
 * raw - dark is exact in float64 and the device decides with one float64 fused
 * multiply-add; otherwise raw - dark is split exactly into two float64 terms
 * and pixels whose estimate lies within rounding of the threshold are decided
 * from an exact expansion of the five-term sum.  Counts are exact either way.
 */
#ifndef RTC_H
#define RTC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RTC_ABI_VERSION 1u

typedef struct rtc_ctx rtc_ctx;

typedef enum {
  RTC_OK = 0,
  RTC_E_ARG = -1,          /* invalid argument, size or pointer */
  RTC_E_STATE = -2,        /* call out of order (e.g. a frame before both loads) */
  RTC_E_NOMEM = -3,        /* host or device allocation failed */
  RTC_E_DEVICE = -4,       /* HIP runtime error or no usable device */
  RTC_E_NONFINITE = -5,    /* NaN/Inf in calibration, threshold, matrix or gains */
  RTC_E_UNSUPPORTED = -6   /* valid request this build does not implement */
} rtc_status;

/* Threshold application (Figure 3 (a)); the paper does not fix the rule.
 * x = (raw - dark) * flat is the calibrated pixel.  The centroid of a
 * subaperture is 0 (minus its reference slopes) unless the sum of its v is
 * positive; in the thresholded modes that is exactly when a pixel is above.
 * Counts report the pixels with x > T in every mode. */
typedef enum {
  RTC_THR_NONE = 0,        /* v = x for every pixel (no threshold applied) */
  RTC_THR_SUBTRACT = 1,    /* v = x - T if x > T else 0 (default) */
  RTC_THR_ZERO = 2         /* v = x     if x > T else 0 */
} rtc_thr_mode;

/* Storage type of the control matrix.  Section 2.3.4 stores it as IEEE
 * binary16 to halve the bytes the bandwidth-bound reconstruction reads and
 * converts each value to 32 bits before the multiply-accumulate; the same is
 * offered for bfloat16 and OCP FP8 E4M3 (e4m3fn).  Reduced formats carry one
 * float32 scale per matrix row:
 *   s_r = 2^e_r, e_r the smallest integer with max_j |R_rj| / 2^e_r <= 2^E
 *         (E = 15 binary16, 0 bfloat16, 8 E4M3), clamped to [-126, 127];
 *         e_r = 0 for an all-zero row;
 *   code  = R_rj / s_r rounded to the nearest value of the format, ties to
 *           the even significand, sign kept on zero (no overflow is possible);
 *   value = decode(code) * s_r; products and sums are float32.
 * Slopes, the integrator and its state stay float32. */
typedef enum {
  RTC_CM_F32 = 0,
  RTC_CM_F16 = 1,
  RTC_CM_BF16 = 2,
  RTC_CM_FP8E4M3 = 3
} rtc_cm_dtype;

typedef struct {
  uint32_t abi_version;        /* must equal RTC_ABI_VERSION */
  int32_t n_sub_x, n_sub_y;    /* subaperture grid, 1..4096 each */
  int32_t n_pix;               /* pixels per subaperture side, 1..32; frame is
                                  H = n_sub_y*n_pix rows x W = n_sub_x*n_pix cols,
                                  H*W < 2^31 */
  const uint8_t *subap_mask;   /* host [n_sub_y][n_sub_x] row-major, nonzero =
                                  active; copied.  Active subapertures are
                                  numbered k = 0..n_valid-1 row-major; k covers
                                  rows [sy*n_pix, +n_pix), cols [sx*n_pix, +n_pix) */
  int32_t n_act;               /* actuators = rows of the control matrix, 1..2^20 */
  int32_t thr_mode;            /* rtc_thr_mode */
  int32_t cm_dtype;            /* rtc_cm_dtype of the stored control matrix */
  float gain, leak;            /* integrator g and leak lambda (1 = pure integrator) */
  float cmd_min, cmd_max;      /* clamp, cmd_min <= cmd_max; +-INFINITY = no clamp */
  int32_t device;              /* HIP device ordinal */
} rtc_config;

/* Creates a context on cfg->device: validates cfg, copies the mask, builds the
 * subaperture index map and allocates the per-frame device buffers.  The
 * integrator state starts at 0.  *out is set only on RTC_OK.
 * Errors: RTC_E_ARG (bad sizes, NULL, no active subaperture, wrong ABI
 * version, unknown thr_mode), RTC_E_NONFINITE (gain/leak/clamp NaN or
 * gain/leak infinite), RTC_E_UNSUPPORTED (reduced-precision matrix with more
 * than 2^24 16-byte chunks per row), RTC_E_DEVICE (no such device),
 * RTC_E_NOMEM. */
rtc_status rtc_init(const rtc_config *cfg, rtc_ctx **out);

/* Several wavefront sensors reconstructed together (the multi-WFS systems of
 * the paper's outlook, Section 3.4.1): each sensor has its own grid, pixels
 * per subaperture and mask; one control matrix maps the concatenated slope
 * vector to n_act actuators.
 *  - Frame set: the sensors' frames back to back, sensor w's H_w x W_w
 *    uint16 frame (H_w = n_sub_y*n_pix, W_w = n_sub_x*n_pix, row-major)
 *    starting at element F_w = sum over v < w of H_v*W_v; the frame set has
 *    rtc_frame_elems() elements and must be < 2^31.  Every frame argument of
 *    the frame calls points to such a set (frame_stride >= rtc_frame_elems).
 *  - Subapertures are numbered sensor by sensor, row-major within a sensor.
 *  - Slope vector: for each sensor in order, its x slopes then its y slopes
 *    (each sensor laid out as Figure 3 (b)); 2*n_valid in total.
 *  - Calibration maps and thresholds follow the same sensor order
 *    (rtc_load_calib_multi).
 * A single-sensor rtc_init is the n_wfs = 1 case of this. */
typedef struct {
  int32_t n_sub_x, n_sub_y;    /* subaperture grid, 1..4096 each */
  int32_t n_pix;               /* pixels per subaperture side, 1..32 */
  const uint8_t *subap_mask;   /* host [n_sub_y][n_sub_x], nonzero = active; copied */
} rtc_wfs;

typedef struct {
  uint32_t abi_version;        /* must equal RTC_ABI_VERSION */
  int32_t n_wfs;               /* 1..64 */
  const rtc_wfs *wfs;          /* host [n_wfs]; copied */
  int32_t n_act;               /* as in rtc_config */
  int32_t thr_mode;
  int32_t cm_dtype;
  float gain, leak;
  float cmd_min, cmd_max;
  int32_t device;
} rtc_multi_config;

/* As rtc_init for several sensors.  Errors as rtc_init, plus RTC_E_ARG for
 * n_wfs outside 1..64, a NULL sensor array or a frame set of 2^31 or more
 * elements. */
rtc_status rtc_init_multi(const rtc_multi_config *cfg, rtc_ctx **out);

/* Elements of one frame set (sum of H_w*W_w; H*W for one sensor), -1 if c NULL. */
int64_t rtc_frame_elems(const rtc_ctx *c);

/* Loads the pixel calibration (Figure 3 (a)): host float32 dark and flat maps
 * [H][W] row-major (flat multiplies: it holds inverse pixel gains), threshold T
 * (finite, >= 0, ADU after flat-fielding), and optional reference slopes
 * ref_slopes [2*n_valid] (x block then y block; NULL = 0) subtracted from the
 * centroids.  Only the active subapertures' pixels are read (and checked),
 * re-laid out per subaperture; other pixels of the maps are ignored.
 * Replaces a previous calibration after synchronising the device.
 * Any finite dark and flat are accepted (see the threshold decision above).
 * Errors: RTC_E_ARG (NULL maps, T < 0), RTC_E_NONFINITE, RTC_E_DEVICE,
 * RTC_E_NOMEM. */
/* rtc_load_calib on a multi-sensor context applies the one threshold to every
 * sensor; dark and flat are laid out as a frame set. */
rtc_status rtc_load_calib(rtc_ctx *c, const float *dark, const float *flat, float threshold,
                          const float *ref_slopes);

/* Multi-sensor calibration: dark and flat as frame sets (rtc_frame_elems
 * floats each), thresholds [n_wfs] (one per sensor, each finite and >= 0),
 * ref_slopes [2*n_valid] or NULL.  Same checks and errors as rtc_load_calib. */
rtc_status rtc_load_calib_multi(rtc_ctx *c, const float *dark, const float *flat, const float *thresholds,
                                const float *ref_slopes);

/* Loads the control matrix R (Section 1.1.1; Figure 3 (c)): host float32,
 * row-major [n_act][ld], row r holds the weights of actuator r over the slope
 * vector (x block then y block); n_slopes must equal 2*n_valid, ld >= n_slopes.
 * It is stored in the context's cm_dtype (encoded on the host as described at
 * rtc_cm_dtype), rows zero-padded to 16-byte multiples.  Replaces a previous
 * matrix (synchronises the device).
 * Errors: RTC_E_ARG (sizes, NULL), RTC_E_NONFINITE, RTC_E_DEVICE, RTC_E_NOMEM. */
rtc_status rtc_load_cmat(rtc_ctx *c, const float *R, int32_t n_act, int32_t n_slopes, int64_t ld);

/* Host-only encoder of the reduced storage formats (no device needed): codes
 * [n_rows][n_cols] (2 bytes per element for F16/BF16, 1 for FP8E4M3) and
 * scales [n_rows] of the float32 rows R [n_rows][ld], exactly as
 * rtc_load_cmat stores them.  Errors: RTC_E_ARG (cm_dtype F32 or unknown,
 * NULL, sizes), RTC_E_NONFINITE. */
rtc_status rtc_encode_cmat(int32_t cm_dtype, const float *R, int32_t n_rows, int32_t n_cols, int64_t ld,
                           void *codes, float *scales);

/* One frame (steps (a)-(d)) on a device uint16 frame d_pixels [H][W] row-major.
 * Writes the new commands c_k to d_cmd [n_act] (float32, device) and advances
 * the integrator state.  Optional device outputs (NULL = not written):
 * d_slopes [2*n_valid] float32, d_recon [n_act] float32 (a_k = R s_k),
 * d_counts [n_valid] int32 (pixels above threshold per subaperture).
 * Errors: RTC_E_STATE (calibration or matrix not loaded), RTC_E_ARG (NULL
 * pixels/cmd), RTC_E_DEVICE (launch failure). */
rtc_status rtc_frame(rtc_ctx *c, const uint16_t *d_pixels, float *d_cmd, float *d_slopes,
                     float *d_recon, int32_t *d_counts, void *hip_stream);

/* n_frames frames in order, as n_frames calls of rtc_frame: frame f reads
 * d_pixels + f*frame_stride (elements, >= H*W) and writes row f of each output:
 * d_cmd [n_frames][n_act] (required), d_slopes [n_frames][2*n_valid],
 * d_recon [n_frames][n_act], d_counts [n_frames][n_valid] (nullable).
 * d_ts (nullable) [n_frames][2] uint64 device wall-clock ticks: [0] when the
 * first calibration workgroup of the frame starts, [1] after the last
 * reconstruction workgroup's results are visible device-wide; the tick rate is
 * rtc_wall_clock_khz().  The integrator state carries across frames.
 * Errors: as rtc_frame, plus RTC_E_ARG for n_frames < 0 or a short stride. */
rtc_status rtc_frame_batch(rtc_ctx *c, int32_t n_frames, const uint16_t *d_pixels,
                           int64_t frame_stride, float *d_cmd, float *d_slopes, float *d_recon,
                           int32_t *d_counts, uint64_t *d_ts, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, fixed-memory serving loops, harnesses that forbid hipMalloc):
 * rtc_frame_batch with the same arguments, results and errors, except that
 * its kernels take every scratch buffer (the slope vectors, split-K partial
 * vectors, completion counter, abort flag and barrier words) from a static
 * device array of the library (4 MiB, one copy per device, held until the
 * process ends) and the call allocates nothing.  The context's device address
 * of the array is resolved by rtc_init.  RTC_FRAMES_HORIZONTAL contexts run
 * the persistent row split here (the horizontal message buffer does not fit).
 * Needs 4 (2 xl + sl + k_split n_act) + 155648 <= 4194304 bytes, with xl =
 * 2 n_valid rounded up to 1024 and sl = 2 n_valid rounded up to 16 (each term
 * then to 64 floats): RTC_E_UNSUPPORTED beyond that, and for device ordinals
 * above 63.  Every such call on one device shares the array, and a call starts
 * by clearing it: calls that overlap on one device (other streams, other
 * contexts, other host threads) race and give undefined results.  A bounded
 * wait that expires raises the context's own flag (rtc_sync_check). */
rtc_status rtc_frame_batch_noalloc(rtc_ctx *c, int32_t n_frames, const uint16_t *d_pixels,
                                   int64_t frame_stride, float *d_cmd, float *d_slopes, float *d_recon,
                                   int32_t *d_counts, uint64_t *d_ts, void *hip_stream);

/* Host-paced frames: the latency of Section 3 (from a frame's arrival to its
 * commands being ready) measured with frames arriving at a fixed rate, the
 * release and completion signalled through spin-waited flags (Section
 * 2.3.2).  Runs a persistent batch (RTC_FRAMES_PERSISTENT required) of
 * n_frames frames, arguments and outputs as rtc_frame_batch, in which frame k
 * starts only once the calling thread releases it, at t0 + k * period_us on
 * the host's CLOCK_MONOTONIC_RAW (busy-waited; t0 = one period after the launch):
 * the thread writes the frame's number to a word of coherent host memory,
 * which workgroup 0 polls and relays to the other workgroups.  The commands
 * of these frames are stored at system scope; the last workgroup to store
 * frame k's commands writes its number to a second host word, on which the
 * thread spins.  h_release_ns[k] and h_done_ns[k] (host arrays, nullable)
 * receive the host times of the release and of the completion being seen, in
 * ns from t0.  Blocks until the batch has ended.  The two words (256 bytes of
 * pinned host memory) are allocated on the first call.
 * Errors: RTC_E_STATE (other frame modes, loads missing, undefined state),
 * RTC_E_ARG (n_frames < 0, NULL pixels/cmd, short stride, period_us not in
 * (0, 1e7]), RTC_E_UNSUPPORTED (tiles wider than 16 pixels, slope vectors
 * long enough for slope panels, darks outside {0} U [2^-13, 2^24)),
 * RTC_E_DEVICE (launch failure, or a frame not complete within 100 periods
 * and at least 100 ms: the remaining frames are then released at once, the
 * batch ends and rtc_sync_check reports the expired wait if there was one). */
rtc_status rtc_paced_batch(rtc_ctx *c, int32_t n_frames, const uint16_t *d_pixels, int64_t frame_stride,
                           float *d_cmd, float *d_slopes, float *d_recon, int32_t *d_counts, uint64_t *d_ts,
                           double period_us, int64_t *h_release_ns, int64_t *h_done_ns, void *hip_stream);

/* Steps (a)-(b) alone: calibration and centre-of-gravity slopes of one frame
 * into d_slopes [2*n_valid] (required) and d_counts [n_valid] (nullable).
 * Leaves the integrator state untouched.  Needs the calibration (RTC_E_STATE). */
rtc_status rtc_calibrate_centroid(rtc_ctx *c, const uint16_t *d_pixels, float *d_slopes,
                                  int32_t *d_counts, void *hip_stream);

/* Steps (c)-(d) alone from a caller slope vector d_slopes [2*n_valid] (device
 * float32): a = R s, then the integrator; writes d_cmd [n_act], optional
 * d_recon [n_act].  Needs the control matrix (RTC_E_STATE). */
rtc_status rtc_reconstruct_integrate(rtc_ctx *c, const float *d_slopes, float *d_cmd,
                                     float *d_recon, void *hip_stream);

/* Launch shape of the reconstruction (step (c)), for tuning.  Two kernels:
 *  kernel = RTC_MVM_ROWBLOCK (default): workgroup b owns a contiguous range of
 *    actuator rows; its `waves` wavefronts (8 or 16) split the slope vector and
 *    keep their slice in registers and decode the stored format there;
 *    `rows_per_batch` rows (1..8) are streamed per batch; `blocks` workgroups
 *    (0 = one per compute unit).  A float32 slope vector longer than the
 *    wavefronts' registers hold falls back to the streamed kernel; reduced
 *    formats widen to 16 wavefronts.
 *  kernel = RTC_MVM_STREAMED (float32 matrices only; RTC_E_UNSUPPORTED for
 *    the others): each wavefront streams `rows_per_wave` (1, 2, 4)
 *    rows against the slope vector staged in LDS, with `unroll` (2, 4, 8; 8
 *    only with rows_per_wave <= 2) 16-byte loads per row in flight, and the
 *    slope dimension split into `k_split` (1..64) partitions whose partial
 *    actuator vectors are summed in a fixed pairwise-tree order (the paper's
 *    tree vector addition, Section 2.3.5).  k_split is raised automatically
 *    when a partition's slopes would not fit 64 KiB of LDS.
 * Results of every shape agree within float32 rounding and each shape is
 * run-to-run deterministic (no floating-point atomics).
 * Default: {RTC_MVM_ROWBLOCK, k_split 1, rows_per_wave 2, unroll 4, blocks 0,
 * waves 8}, the fastest shape measured at the ELT size. */
typedef enum { RTC_MVM_ROWBLOCK = 0, RTC_MVM_STREAMED = 1 } rtc_mvm_kernel;

typedef struct {
  int32_t kernel;          /* rtc_mvm_kernel */
  int32_t k_split;         /* streamed */
  int32_t rows_per_wave;   /* streamed: rows per wavefront; row-block: rows per batch */
  int32_t unroll;          /* streamed */
  int32_t blocks;          /* row-block: workgroups, 0 = compute-unit count */
  int32_t waves;           /* row-block: wavefronts per workgroup, 8 or 16 */
} rtc_mvm_tuning;

rtc_status rtc_set_mvm_tuning(rtc_ctx *c, const rtc_mvm_tuning *t);
rtc_status rtc_get_mvm_tuning(const rtc_ctx *c, rtc_mvm_tuning *t);

/* How rtc_frame_batch runs its frames.
 *  RTC_FRAMES_PER_LAUNCH (default): two kernel launches per frame.
 *  RTC_FRAMES_PERSISTENT: one cooperative launch for the whole batch.  Each
 *    workgroup (one per compute unit) calibrates its share of the
 *    subapertures of frame f, waits at a grid barrier for all slopes of frame
 *    f, then reconstructs and integrates its own actuator rows; the rows'
 *    integrator state stays on chip across frames.  This replaces the paper's
 *    spin-locks and volatile flags (Section 2.3.2) with one device-wide
 *    counter per frame.  Every wait is bounded by spin_limit polls (0 = the
 *    default, about 0.1-0.3 s); when one expires the batch winds down, its
 *    remaining frames are not processed and rtc_sync_check reports it.
 *    Shapes the persistent kernel does not cover (more than 512 actuator rows
 *    per compute unit, slope slices beyond its registers, a grid that cannot
 *    be co-resident, a calibration with a dark outside {0} U [2^-13, 2^24) in
 *    magnitude) run per launch instead.  The arithmetic and its order
 *    are those of the per-launch mode with the row-block kernel, 8 wavefronts
 *    and the same workgroup count, so results are bitwise identical to it.
 *  RTC_FRAMES_HORIZONTAL: one cooperative launch of 256 workgroups of 256
 *    threads for the whole batch, in the paper's horizontal processing
 *    strategy (Section 2.2, Figure 5; the partial-vector sum of Section
 *    2.3.5): workgroup b calibrates subapertures [b n_valid / 256,
 *    (b+1) n_valid / 256) and multiplies their slopes into its own columns of
 *    the control matrix for every actuator row -- columns that stay in its
 *    registers and LDS for the whole batch -- giving a partial actuator
 *    vector; after one grid barrier per frame, workgroup o adds the 256
 *    partial vectors of its actuator rows [o q + min(o, r), (o+1) q +
 *    min(o+1, r)) (q = n_act / 256, r = n_act mod 256) in a fixed order and
 *    applies the integrator.  No slope leaves the workgroup that computed it.
 *    The matrix is re-laid out on the device for this split when the mode is
 *    set or a matrix is loaded in it (about 1.07 x the stored matrix, plus a
 *    16.8 MB message buffer).  Needs 256 compute units and shapes whose
 *    columns and rows fit on chip (at most 32 slope columns per workgroup and,
 *    for the float32 ELT shape, at most 18 actuator rows per workgroup and
 *    tiles of at most 10 pixels): RTC_E_UNSUPPORTED otherwise.  Batches whose
 *    frames the kernel cannot read as pixel pairs (an odd frame stride or an
 *    unaligned pointer) or whose calibration has a dark outside
 *    {0} U [2^-13, 2^24) run per launch.  Results equal the other modes within
 *    float32 rounding (the sums run in another fixed order) and are
 *    run-to-run bitwise deterministic.  rtc_set_trace stamps for this mode:
 *    [0] frame start, [1] slopes in LDS, [4] partial vector published, [6]
 *    own stores complete, [7] arrival counted, [2] barrier passed, [3] partial
 *    vectors loaded, [5] commands written. */
typedef enum { RTC_FRAMES_PER_LAUNCH = 0, RTC_FRAMES_PERSISTENT = 1, RTC_FRAMES_HORIZONTAL = 2 } rtc_frame_mode;

rtc_status rtc_set_frame_mode(rtc_ctx *c, int32_t mode, int32_t spin_limit);
/* Current frame mode into *mode. */
rtc_status rtc_get_frame_mode(const rtc_ctx *c, int32_t *mode);

/* Stage tracing of persistent batches: when set, each persistent batch writes
 * for its frames f < max_frames and its workgroups g < n_groups the device
 * wall-clock stamps (rtc_wall_clock_khz ticks) at
 * d_trace[f][g][0..7] = frame start, own slopes issued, frame barrier
 * passed, slope slices loaded, partial sums done, commands written, own
 * stores complete (barrier entry), own arrival counted.  Entries of
 * workgroups the batch does not launch stay untouched.
 * d_trace is a caller-owned device buffer of max_frames * n_groups * 8
 * uint64 that must stay valid while batches run; max_frames = 0 turns
 * tracing off; n_groups must be in [1, 4096] when max_frames > 0. */
rtc_status rtc_set_trace(rtc_ctx *c, uint64_t *d_trace, int32_t max_frames, int32_t n_groups);

/* Graph replay: records rtc_frame_batch with these arguments, in the
 * context's current frame mode and tuning, into a HIP graph held by the
 * context (replacing a previous one; the recording itself runs nothing), and
 * rtc_graph_launch replays it on hip_stream.  Every replay processes the same
 * frames into the same buffers, continuing from the integrator state that
 * the previous replay or frame call left, exactly as the recorded call
 * would.  The buffers must stay valid while the graph exists (until the next
 * capture or rtc_destroy).  Counters are cleared by kernels, so the graph
 * holds no memset nodes.  Errors: as rtc_frame_batch; RTC_E_UNSUPPORTED when
 * the runtime cannot record the frame mode's launches (nothing is recorded);
 * rtc_graph_launch without a graph: RTC_E_STATE. */
rtc_status rtc_graph_capture(rtc_ctx *c, int32_t n_frames, const uint16_t *d_pixels, int64_t frame_stride,
                             float *d_cmd, float *d_slopes, float *d_recon, int32_t *d_counts, uint64_t *d_ts);
rtc_status rtc_graph_launch(rtc_ctx *c, void *hip_stream);

/* Autotuner: one timed candidate of rtc_autotune. */
typedef struct {
  int32_t frame_mode;          /* rtc_frame_mode */
  rtc_mvm_tuning tuning;
  float us_per_frame;          /* mean over the timed frames (HIP events); < 0: the candidate failed */
} rtc_tune_result;

/* Times n_frames frames (after n_frames/4 + 1 untimed ones) of d_pixels
 * (frame_stride apart; outputs to d_cmd, n_frames * n_act floats) on
 * hip_stream for every candidate: persistent with 1x and 3/4x the compute
 * units; per launch with the row-block kernel (8 and 16 wavefronts, 1, 2 and
 * 4 rows per batch, 1x and 2x the compute units) and, for float32 matrices,
 * the streamed kernel with 1, 2 and 4 slope partitions.  Sets the fastest
 * frame mode and tuning on the context and restores the integrator state it
 * found.  Up to max_results results go to results (may be NULL); *n_results
 * (may be NULL) gets the number of candidates.  Synchronous.  Errors: as
 * rtc_frame_batch, RTC_E_ARG for n_frames < 1. */
rtc_status rtc_autotune(rtc_ctx *c, int32_t n_frames, const uint16_t *d_pixels, int64_t frame_stride,
                        float *d_cmd, rtc_tune_result *results, int32_t max_results, int32_t *n_results,
                        void *hip_stream);

/* Row split of persistent batches (an unequal allocation of the
 * reconstruction's rows to workgroups, in the spirit of the unequal
 * allocation of Section 2.3.6: equal shares finish at different times when
 * the workers are not equally fast).  With row_start set, workgroup b of a
 * persistent launch of G workgroups owns the contiguous actuator rows
 * [row_start[b], row_start[b+1]) instead of [b n_act / G, (b+1) n_act / G).
 * row_start: host array of G + 1 int32 with row_start[0] = 0,
 * row_start[G] = n_act, every share >= 1 and <= 512 rows; copied.  The
 * split applies to persistent launches whose grid is G workgroups (the
 * compute-unit count, or the tuning's block count, capped at n_act); other
 * launches keep the equal split.  Results are bitwise those of the equal
 * split (each row's sum does not depend on the workgroup computing it).
 * G = 0 or row_start = NULL restores the equal split.  Waits until the
 * device is idle (a running batch may read the split); a recorded graph is
 * discarded (its launch shape may no longer fit).  Errors: RTC_E_ARG for a
 * malformed split or G outside [0, 1024]. */
rtc_status rtc_set_row_split(rtc_ctx *c, int32_t G, const int32_t *row_start);
/* The current split into row_start (host, room for G + 1 entries; may be
 * NULL) and its grid into *G (0 = equal split). */
rtc_status rtc_get_row_split(const rtc_ctx *c, int32_t *G, int32_t *row_start, int32_t capacity);

/* Measured row split for the current persistent tuning: traces a batch of
 * n_frames frames of d_pixels (frame_stride apart; outputs to d_cmd,
 * n_frames * n_act floats) with the equal split, takes each workgroup's
 * median time of its partial sums over the last three quarters of the
 * frames, gives every workgroup rows in proportion to its measured rows per
 * second (largest remainders, every share >= 1 and <= 512), times a batch
 * with both splits (HIP events, after n_frames/4 + 1 untimed frames) and
 * keeps the faster (the traced batch is not one of the timed ones).
 * *us_equal and *us_split (may be NULL) get the mean frame times of the two.
 * The integrator state and the trace setting are restored; a recorded graph
 * is discarded.  Synchronous; allocates a trace buffer for the measurement.
 * Errors: as rtc_frame_batch; RTC_E_STATE when the context is not in the
 * persistent frame mode or the persistent launch is not supported for its
 * shape; RTC_E_ARG for n_frames < 4. */
rtc_status rtc_balance_rows(rtc_ctx *c, int32_t n_frames, const uint16_t *d_pixels, int64_t frame_stride,
                            float *d_cmd, float *us_equal, float *us_split, void *hip_stream);

/* ---- Pixel-stream processing (Section 2.3.6 and Figure 6; the latency
 * measurements of Section 3.2, Figures 11 and 12) ----
 *
 * The frame is processed while its pixels arrive.  A camera emulator inside
 * the launch lands the rows of each frame in a two-slot ring held by the
 * context: rows of frame f land uniformly over readout_us from the frame's
 * scheduled start f * frame_period_us (after a short lead), in packets of
 * rows_per_packet rows, each packet followed by a landed-row count.  The
 * other workgroups are workers (the paper's processing threads, horizontal
 * strategy): worker b owns a contiguous run of subapertures in arrival
 * order, and as soon as the rows a group of them needs have landed it
 * calibrates and centroids them and multiplies their slopes into the matching
 * columns of the control matrix, accumulating a partial actuator vector.  The
 * P partial vectors are added per actuator in worker order by the owners --
 * the first half of the workers, whose own subapertures land early -- each
 * vector as soon as it is published (the vector addition of Section 2.3.5
 * and Figure 5 becomes a running sum that keeps pace with the arrivals), and
 * the integrator is applied.  Latency, as in the paper, is the time from the
 * last pixel of a frame landing to its last command being written.
 *
 * Subaperture allocation: counts decrease linearly from the first worker to
 * the last with first / last = alloc_ratio (1 = equal shares, Figure 6 (c);
 * > 1 = unequal, Figure 6 (d)), so workers whose pixels arrive last have the
 * least to do after the last pixel.  full_frame = 1 makes every subaperture
 * wait for the whole frame (no pixel-stream processing) for comparison.
 *
 * Tail: the subapertures of the last tail_rows subaperture rows (at most 64)
 * are left out of the allocation; instead every owner calibrates them itself
 * once their rows land and multiplies their slopes into its own actuator rows
 * (a row split of those columns, from LDS), so that after the last pixel no
 * partial vector has to travel between workgroups.
 * Results do not depend on the allocation or the tail beyond float32
 * rounding order. */
typedef struct {
  int32_t n_workers;           /* worker workgroups, 0 = compute units - 1; one more runs the camera */
  int32_t full_frame;          /* 0 or 1 */
  double alloc_ratio;          /* subapertures of the first worker / of the last, in [1, 1000] */
  double frame_period_us;      /* camera frame period, (0, 1e6] */
  double readout_us;           /* (0, frame_period_us] */
  int32_t rows_per_packet;     /* >= 1 */
  int32_t wait_limit_us;       /* a wait gives up after this long; 0 = 2 frame periods + 50 ms */
  int32_t tail_rows;           /* subaperture rows at the bottom of the frame taken by every worker, 0..n_sub_y */
  int32_t reserved;            /* 0 */
} rtc_pipe_config;

/* Linearly decreasing allocation (host only, no device): counts[b] for b <
 * n_workers, summing to n_subaps.  Target shares are proportional to
 * w_b = ratio + (1 - ratio) b / (n_workers - 1) (w = 1 for one worker); each
 * count is the floor of its share, and the remaining subapertures go one each
 * to the largest fractional parts (ties to the lower index).  Errors:
 * RTC_E_ARG for n_subaps < 0, n_workers < 1, ratio outside [1, 1000] or NaN,
 * NULL counts. */
rtc_status rtc_pipe_allocation(int32_t n_subaps, int32_t n_workers, double ratio, int32_t *counts);

/* Prepares pixel-stream processing of a single-sensor context: copies the
 * stored control matrix column-major (x and y columns of each subaperture
 * adjacent, any storage format), the allocation and the rows each
 * subaperture needs (its last pixel row + 1, or every row with full_frame),
 * and allocates the ring, partial vectors and counters.  Call after
 * rtc_load_cmat, and again after each new matrix.  Synchronous.  Errors:
 * RTC_E_STATE without a matrix; RTC_E_ARG for a config out of range;
 * RTC_E_UNSUPPORTED for several sensors, n_act > 8192, more than 64 actuator
 * rows per worker, more than 64 tail subapertures or an odd frame size;
 * RTC_E_NOMEM / RTC_E_DEVICE. */
rtc_status rtc_pipe_setup(rtc_ctx *c, const rtc_pipe_config *cfg);

/* Shape chosen by rtc_pipe_setup (any pointer may be NULL): workers, matrix
 * columns per worker kept in LDS, image rows, most subapertures of a worker,
 * tail subapertures, owners (workers 0..n_owners-1 hold the actuator rows). */
rtc_status rtc_pipe_info(const rtc_ctx *c, int32_t *n_workers, int32_t *lds_cols, int32_t *image_rows,
                         int32_t *max_subaps, int32_t *n_tail, int32_t *n_owners);

/* Runs n_frames frames through the camera emulator and the workers in one
 * launch on hip_stream (asynchronous).  d_frames: n_frames source frames,
 * frame_stride (even, >= rtc_frame_elems) elements apart, 4-byte aligned;
 * they are copied row by row into the ring as they "arrive".  Outputs as
 * rtc_frame_batch (d_cmd [n_frames][n_act]; d_slopes, d_recon, d_counts
 * nullable).  Time stamps (device wall clock, rtc_wall_clock_khz ticks,
 * nullable): d_cam_ts [n_frames][4] = scheduled frame start, first packet
 * landed, last packet landed (the last pixel), largest delay of a packet
 * behind its schedule; d_worker_ts [n_frames][n_workers][2] = worker's
 * partial vector published, worker done with the frame (an owner: its
 * actuator rows integrated and stored).  The integrator
 * state carries across calls and frame modes.  A wait that exceeds
 * wait_limit_us gives up, and the batch stops early; rtc_sync_check reports
 * it.  Errors: RTC_E_STATE before rtc_pipe_setup or after a new
 * matrix; RTC_E_ARG for bad arguments; RTC_E_UNSUPPORTED when a dark of the
 * calibration is outside {0} U [2^-13, 2^24) in magnitude (the exact threshold
 * path runs in the per-launch calibration only); RTC_E_DEVICE when the launch
 * fails. */
rtc_status rtc_pipe_run(rtc_ctx *c, int32_t n_frames, const uint16_t *d_frames, int64_t frame_stride,
                        float *d_cmd, float *d_slopes, float *d_recon, int32_t *d_counts, uint64_t *d_cam_ts,
                        uint64_t *d_worker_ts, void *hip_stream);

/* Synchronises the device and reports RTC_E_DEVICE if a persistent or
 * pixel-stream batch gave up at a bounded wait since the last check (the flag
 * is then cleared).  In such a batch the workgroup whose wait expired computes
 * neither that frame nor later ones, so the commands of those frames are not
 * written and each actuator row's integrator state stops at the last frame its
 * workgroup completed: the state is undefined.  After this report rtc_frame,
 * rtc_frame_batch, rtc_reconstruct_integrate, rtc_graph_launch and
 * rtc_pipe_run fail with RTC_E_STATE until rtc_reset or rtc_set_state. */
rtc_status rtc_sync_check(rtc_ctx *c);

/* Integrator state: reset to 0, synchronous host copy out / in (n_act floats,
 * all finite for set).  They synchronise the device first. */
rtc_status rtc_reset(rtc_ctx *c);
rtc_status rtc_get_state(rtc_ctx *c, float *h_cmd);
rtc_status rtc_set_state(rtc_ctx *c, const float *h_cmd);

/* Sizes: active subapertures (= popcount of the mask), actuators. -1 if c NULL. */
int32_t rtc_n_valid(const rtc_ctx *c);
int32_t rtc_n_act(const rtc_ctx *c);

/* Frequency of the device wall clock used by rtc_frame_batch time stamps, kHz. */
rtc_status rtc_wall_clock_khz(rtc_ctx *c, int64_t *khz);

/* Bandwidth probes on the context's device (roofline calibration):
 * copy n_bytes (multiple of 16) from d_src to d_dst, or read n_bytes of d_src
 * and write one float checksum to d_out.  Asynchronous on hip_stream. */
rtc_status rtc_probe_copy(rtc_ctx *c, const void *d_src, void *d_dst, int64_t n_bytes,
                          void *hip_stream);
rtc_status rtc_probe_read(rtc_ctx *c, const void *d_src, int64_t n_bytes, float *d_out,
                          void *hip_stream);

/* Last error text of c (context-local), or of the calling thread's last failed
 * rtc_init when c is NULL.  Valid until the next call on the same context. */
const char *rtc_error_string(const rtc_ctx *c);

/* ABI version the library was built with (RTC_ABI_VERSION). */
uint32_t rtc_abi_version(void);

/* Frees the context and its device memory (synchronises its device first).
 * NULL is ignored. */
void rtc_destroy(rtc_ctx *c);

#ifdef __cplusplus
}
#endif

#endif /* RTC_H */
