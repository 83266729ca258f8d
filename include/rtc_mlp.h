/* rtc_mlp.h -- C ABI of the learned predictor of the real-time controller.
 *
 * A two-layer perceptron forecasts the next frame's modal coefficients of the
 * pseudo-open-loop slopes from the last frames' coefficients (the servo lag of
 * the integrator of Section 2.1 / Figure 3 (d) is what it is meant to cancel):
 *     Z1 = X W1^T + b1,  H = GELU(Z1),  Y = H W2^T + b2,
 * X [batch][n_in], W1 [n_hidden][n_in], W2 [n_out][n_hidden].  Products take
 * bfloat16 operands (X, W1, W2, H and the backward gradients are rounded to
 * bfloat16 to nearest even where they enter a product) with float32
 * accumulation on the matrix cores; biases, GELU, loss and Adam are float32;
 * master parameters are float32.  GELU(z) = z Phi(z) with the exact normal
 * CDF.  Loss = mean over batch and outputs of (Y - T)^2.
 *
 * Conventions as rtc.h: host arrays are copied; device pointers are
 * caller-owned; calls are asynchronous on the given HIP stream unless stated;
 * every call returns an rtc_status and changes nothing on error.
 */
#ifndef RTC_MLP_H
#define RTC_MLP_H

#include <stdint.h>

#include "rtc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rtc_mlp rtc_mlp;

/* Network of n_in -> n_hidden (GELU) -> n_out for batches up to max_batch on
 * HIP device `device`; parameters start at zero.  Errors: RTC_E_ARG (sizes
 * outside 1..2^16, max_batch outside 1..2^16), RTC_E_DEVICE, RTC_E_NOMEM. */
rtc_status rtc_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t max_batch, int32_t device,
                          rtc_mlp **out);

/* Host float32 parameters: W1 [n_hidden][n_in], b1 [n_hidden], W2 [n_out][n_hidden],
 * b2 [n_out] (all finite; RTC_E_NONFINITE otherwise).  Setting resets the Adam
 * moments.  Both synchronise the device. */
rtc_status rtc_mlp_set_params(rtc_mlp *m, const float *W1, const float *b1, const float *W2, const float *b2);
rtc_status rtc_mlp_get_params(rtc_mlp *m, float *W1, float *b1, float *W2, float *b2);

/* Forward pass: d_y [batch][n_out] = network(d_x [batch][n_in]) (float32 device
 * arrays, row-major).  RTC_E_ARG for batch outside 1..max_batch. */
rtc_status rtc_mlp_forward(rtc_mlp *m, int32_t batch, const float *d_x, float *d_y, void *hip_stream);

/* Forward and backward pass on a batch with targets d_t [batch][n_out]: the
 * loss goes to d_loss (one float, device) and the parameter gradients are kept
 * in the network for rtc_mlp_get_grads / rtc_mlp_adam. */
rtc_status rtc_mlp_loss_grad(rtc_mlp *m, int32_t batch, const float *d_x, const float *d_t, float *d_loss,
                             void *hip_stream);

/* Synchronous host copy of the last gradients (shapes as the parameters). */
rtc_status rtc_mlp_get_grads(rtc_mlp *m, float *dW1, float *db1, float *dW2, float *db2);

/* One Adam step (Kingma & Ba) on the last gradients with bias correction for
 * step number `step` >= 1: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * theta -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps). */
rtc_status rtc_mlp_adam(rtc_mlp *m, float lr, float beta1, float beta2, float eps, int32_t step, void *hip_stream);

void rtc_mlp_destroy(rtc_mlp *m);

/* Predictive feed-forward for the integrator, around a network with
 * n_in = history * n_modes and n_out = n_modes.  Per frame k, with measured
 * slopes r_k and the command c_{k-1} the mirror held while they were taken:
 *   m_k = P r_k + PD c_{k-1}                 pseudo-open-loop modes [n_modes]
 *   window <- last `history` changes (m_k - m_{k-1} - mean) / std
 *   d_k = network(window) * std + mean       forecast change m_{k+1} - m_k
 *                                            (0 until history + 1 frames)
 *   r'_k = r_k + P^T d_k / gain              slopes handed to the integrator
 * where P [n_modes][n_slopes] has orthonormal rows (modes of the slope
 * space), PD = P D [n_modes][n_act] maps commands to their modal slopes, and
 * mean / std normalise the per-frame changes of the modes.
 * The integrator c_k = c_{k-1} + gain R r'_k (rtc_reconstruct_integrate with
 * the same gain) then adds R P^T d_k to its command: the forecast change of the
 * leading modes is applied in the frame it happens instead of one frame
 * later.  With a zero forecast r' = r and the controller is the plain
 * integrator, which is the fallback.  The network is borrowed and must
 * outlive the predictor.  Errors as rtc_mlp_create, RTC_E_ARG for shapes that
 * do not match the network, RTC_E_NONFINITE for non-finite inputs,
 * non-positive std or gain. */
typedef struct rtc_pred rtc_pred;

rtc_status rtc_pred_create(rtc_mlp *net, int32_t history, int32_t n_modes, int32_t n_slopes, int32_t n_act,
                           const float *P, const float *PD, const float *mean, const float *std_, float gain,
                           rtc_pred **out);

/* Empties the history window (synchronous). */
rtc_status rtc_pred_reset(rtc_pred *p);

/* One frame: d_slopes [n_slopes] (r_k), d_cmd_prev [n_act] (c_{k-1}),
 * d_slopes_out [n_slopes] (r'_k; must not alias the inputs); d_modes
 * (nullable) [2][n_modes] receives m_k and the forecast m_k + d_k. */
rtc_status rtc_pred_step(rtc_pred *p, const float *d_slopes, const float *d_cmd_prev, float *d_slopes_out,
                         float *d_modes, void *hip_stream);

/* Predictive frames: n_frames frames of context c, each as rtc_frame_batch
 * runs it in the per-launch mode (calibration and centroids, reconstruction
 * and integrator) with the predictor step of p between them -- r_k measured,
 * c_{k-1} = the context's integrator state, r'_k handed to the
 * reconstruction -- so that c_k = c_{k-1} + gain R r'_k as above.  When the
 * context is in RTC_FRAMES_PERSISTENT mode and the built kernels cover its
 * shape (FP32 matrix, at most 256 actuator rows per workgroup and 4 chunks
 * per lane, tiles of up to 16 pixels, network sizes n_in and n_hid multiples
 * of 4), all frames run in one persistent launch with the step's four
 * phases between the slope exchange and the products, each followed by a
 * grid barrier; the results are bitwise those of the per-launch form, which
 * runs otherwise.  The persistent form records no stage trace
 * (rtc_set_trace).  An expired barrier wait there leaves the context's state
 * undefined (rtc_sync_check) and the predictor's too (rtc_pred_reset).  Frame f
 * reads d_pixels + f * frame_stride (elements, >= one frame) and writes
 * d_cmd [n_frames][n_act] (required) and d_slopes [n_frames][n_slopes]
 * (measured r_k, nullable); d_ts (nullable) [n_frames][2] gets the frame's
 * start (calibration) and end (last command stored) device wall-clock ticks
 * (rtc_wall_clock_khz), as in rtc_frame_batch.  p must have been created for
 * c's slope and actuator counts on c's device and the context's gain.
 * Errors: RTC_E_ARG (sizes, devices, pointers, stride), RTC_E_STATE (loads
 * missing, undefined state), RTC_E_DEVICE (launch failure; the text is in
 * rtc_pred_error_string). */
rtc_status rtc_pred_frame_batch(rtc_ctx *c, rtc_pred *p, int32_t n_frames, const uint16_t *d_pixels,
                                int64_t frame_stride, float *d_cmd, float *d_slopes, uint64_t *d_ts,
                                void *hip_stream);

/* The frame mode the last successful rtc_pred_frame_batch of p ran in:
 * RTC_FRAMES_PERSISTENT (one launch) or RTC_FRAMES_PER_LAUNCH (four step
 * launches between the frame's own); RTC_FRAMES_PER_LAUNCH before any batch.
 * Errors: RTC_E_ARG (NULL argument). */
rtc_status rtc_pred_last_batch_mode(const rtc_pred *p, int32_t *mode);

void rtc_pred_destroy(rtc_pred *p);

/* Last error text of a network / predictor, or of the calling thread's last
 * failed create call when the argument is NULL. */
const char *rtc_mlp_error_string(const rtc_mlp *m);
const char *rtc_pred_error_string(const rtc_pred *p);

#ifdef __cplusplus
}
#endif

#endif /* RTC_MLP_H */
