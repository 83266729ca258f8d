// Internal interface between the predictor's C-ABI host code and its gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtcm {

// C[m][n] = alpha sum_k A(m, k) B(k, n) (+ bias[n]), optional GELU; float32
// accumulation on bfloat16 operands.  A(m, k) = a[m sam + k sak] and
// B(k, n) = b[k sbk + n sbn], read from float32 (rounded to bfloat16 on load)
// or bfloat16 storage (exactly one of the two pointers set per operand).
struct GemmArgs {
  int M, N, K;
  const float *a_f32;
  const uint16_t *a_bf16;
  int64_t sam, sak;
  const float *b_f32;
  const uint16_t *b_bf16;
  int64_t sbk, sbn;
  float alpha;
  const float *bias;   // nullable [N]
  int gelu;            // apply GELU after the bias
  int64_t ldc;
  float *c_pre;        // nullable: value before the GELU
  float *c_f32;        // nullable: result
  uint16_t *c_bf16;    // nullable: result rounded to bfloat16
  float *ws;           // nullable: split-K workspace of ws_len floats (no split without it)
  int64_t ws_len;
};
hipError_t launch_gemm(const GemmArgs &g, hipStream_t st);

hipError_t launch_round_bf16(const float *x, uint16_t *y, int64_t n, hipStream_t st);
hipError_t launch_loss_grad(const float *Y, const float *T, int B, int n, float *dY, uint16_t *dYb, float *row_sq,
                            float *loss, hipStream_t st);
hipError_t launch_gelu_back(const float *dH, const float *Z, float *dZ, uint16_t *dZb, int64_t n, hipStream_t st);
hipError_t launch_col_sum(const float *dZ, int B, int n, float *db, hipStream_t st);
hipError_t launch_adam(float *theta, float *m, float *v, const float *grad, uint16_t *theta_b, int64_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2, hipStream_t st);
// One predictor step (four launches): modes m = P s + (P D) c and their
// history window; with a full window the network (layer 1 with GELU, layer 2)
// and the forecast change d = y std + mean, else d = 0; the feed-forward
// slopes s_out = s + P^T d / gain.  Matrices are float32 rows padded with zeros
// to a multiple of 4 elements (16-byte aligned rows); network weights are the
// bfloat16 copies, inputs rounded to bfloat16 as they are read.
struct PredStepArgs {
  const float *P;        // [n_modes][ldp]
  int64_t ldp;
  const float *PD;       // [n_modes][ldd]
  int64_t ldd;
  const float *PT;       // [n_slopes][ldt]
  int64_t ldt;
  const float *s;        // [n_slopes] measured slopes
  const float *c;        // [n_act] previous commands
  int n_slopes, n_act, n_modes, history, n_in, n_hid;
  int push;              // a previous frame exists (the window takes a change)
  int full;              // the window holds `history` changes (the network runs)
  float *hist;           // [2 history][n_modes] ring of normalised changes: a change goes to slots
                         // pos and pos + history, so slots pos + 1 .. pos + history are the window
  int pos;               // ring slot of this frame's change
  float *m, *m_prev;     // [n_modes]
  const float *mean, *std_, *inv_std;
  const uint16_t *W1;    // [n_hid][n_in]
  const float *b1;
  const uint16_t *W2;    // [n_modes][n_hid]
  const float *b2;
  float *h;              // [n_hid] hidden activations
  float *d;              // [n_modes] forecast change
  float *modes_out;      // nullable [2 n_modes]: m, then m + d
  float *s_out;          // [n_slopes]
  float inv_gain;
};
hipError_t launch_pred_step(const PredStepArgs &a, hipStream_t st);

}  // namespace rtcm
