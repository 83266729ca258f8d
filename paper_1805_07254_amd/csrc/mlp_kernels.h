// Internal interface between the predictor's C-ABI host code and its gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pred_step.h"

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
// deferred (nullable): when the product splits K, leave the sums of the
// partial results (ws[z][M][N], z < *deferred, added in split order) to the
// consumer instead of a second kernel; *deferred = 0 when the result was
// written.  Only for products with alpha = 1 and no GELU, whose consumer
// takes the partials (launch_loss_grad, launch_gelu_back).
hipError_t launch_gemm(const GemmArgs &g, hipStream_t st, int *deferred = nullptr);

hipError_t launch_round_bf16(const float *x, uint16_t *y, int64_t n, hipStream_t st);
// parts, splits > 0: Y = (sum of the splits' partials in split order) + bias,
// as the product's own epilogue would compute it; else Y is read.
hipError_t launch_loss_grad(const float *Y, const float *T, int B, int n, float *dY, uint16_t *dYb, float *row_sq,
                            float *loss, hipStream_t st, const float *parts = nullptr, int splits = 0,
                            const float *bias = nullptr);
// parts, splits > 0: dH = sum of the splits' partials in split order.
hipError_t launch_gelu_back(const float *dH, const float *Z, float *dZ, uint16_t *dZb, int64_t n, hipStream_t st,
                            const float *parts = nullptr, int splits = 0);
hipError_t launch_col_sum(const float *dZ, int B, int n, float *db, hipStream_t st);
// Adam with bias correction on up to kAdamTensors tensors in one launch,
// refreshing each tensor's bfloat16 copy.
constexpr int kAdamTensors = 4;
struct AdamTensor {
  float *theta, *m, *v;
  const float *grad;
  uint16_t *theta_b;   // nullable bfloat16 copy
  int64_t n;
};
hipError_t launch_adam_multi(const AdamTensor *t, int count, float lr, float b1, float b2, float eps, float c1,
                             float c2, hipStream_t st);
// One predictor step in four launches (arguments and arithmetic in
// pred_step.h and pred_device.h).
hipError_t launch_pred_step(const PredStepArgs &a, hipStream_t st);

}  // namespace rtcm
