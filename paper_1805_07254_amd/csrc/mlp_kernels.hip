// gfx950 kernels of the learned predictor: a two-layer perceptron trained and
// run with bfloat16 operands and float32 accumulation.
//
//   gemm_bf16_kernel   C = alpha op(A) op(B) (+ bias) with an optional GELU, on
//                      the 32x32x16 bfloat16 matrix cores; operands are read
//                      with arbitrary element strides, so the forward
//                      (X W^T), weight-gradient (dZ^T X) and input-gradient
//                      (dZ W) products are one kernel
//   elementwise        bfloat16 rounding, loss and its gradient, GELU
//                      derivative, bias gradients, Adam
//   gemv_f32_kernel    y = alpha A x + beta y (modal projection of the
//                      predictor step; one wavefront per row)
//
// Every reduction has a fixed order: results are run-to-run deterministic.
#include "mlp_kernels.h"

namespace rtcm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// bfloat16 of a float, round to nearest even (NaN stays a quiet NaN).
__device__ __forceinline__ uint16_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * z * z);
  return cdf + z * pdf;
}

// ---------------------------------------------------------------------------
// GEMM.  Workgroup = 4 wavefronts computing a 64 x 64 tile of C; wavefront w
// owns the 32 x 32 sub-tile (w / 2, w % 2).  Per K step of 32 the A (64 x 32)
// and B (32 x 64) tiles are staged in LDS as bfloat16 (zero outside the
// matrices), then each wavefront issues two 32x32x16 matrix-core operations.
// Operand layout of the 32x32x16 operation: lane l supplies row (A) or column
// (B) l % 32 and the eight consecutive k = 8 (l / 32) .. 8 (l / 32) + 7; its
// 16 results are column l % 32, rows 8 (v / 4) + 4 (l / 32) + v % 4.
constexpr int kTile = 64, kK = 32, kPad = 8;

__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g) {
  __shared__ uint16_t As[kTile][kK + kPad];        // [m][k]
  __shared__ uint16_t Bs[kTile][kK + kPad];        // [n][k]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0f;

  for (int k0 = 0; k0 < g.K; k0 += kK) {
    // stage: 64 x 32 elements of each operand, 8 per thread
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = r * 256 + tid;
      const int i = e / kK, kk = e % kK;           // i: row of A / column of B within the tile
      const int m = m0 + i, n = n0 + i, k = k0 + kk;
      uint16_t a = 0, b = 0;
      if (m < g.M && k < g.K) {
        const int64_t off = (int64_t)m * g.sam + (int64_t)k * g.sak;
        a = g.a_f32 ? bf16_bits(g.a_f32[off]) : g.a_bf16[off];
      }
      if (n < g.N && k < g.K) {
        const int64_t off = (int64_t)k * g.sbk + (int64_t)n * g.sbn;
        b = g.b_f32 ? bf16_bits(g.b_f32[off]) : g.b_bf16[off];
      }
      As[i][kk] = a;
      Bs[i][kk] = b;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kK; ks += 16) {
      bf16x8 av, bv;
      const int kb = ks + 8 * (lane >> 5);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        av[j] = __builtin_bit_cast(__bf16, As[wm + (lane & 31)][kb + j]);
        bv[j] = __builtin_bit_cast(__bf16, Bs[wn + (lane & 31)][kb + j]);
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
    }
    __syncthreads();
  }

  const int n = n0 + wn + (lane & 31);
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int m = m0 + wm + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    if (m < g.M && n < g.N) {
      float z = g.alpha * acc[v];
      if (g.bias) z += g.bias[n];
      const int64_t o = (int64_t)m * g.ldc + n;
      if (g.c_pre) g.c_pre[o] = z;
      const float y = g.gelu ? gelu(z) : z;
      if (g.c_f32) g.c_f32[o] = y;
      if (g.c_bf16) g.c_bf16[o] = bf16_bits(y);
    }
  }
}

// ---------------------------------------------------------------------------
// elementwise and reductions
__global__ __launch_bounds__(256) void round_bf16_kernel(const float *x, uint16_t *y, int64_t n) {
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) y[i] = bf16_bits(x[i]);
}

// dY = 2 (Y - T) / (B n_out) (float32 and bfloat16) and per-row sums of (Y - T)^2.
__global__ __launch_bounds__(256) void loss_grad_kernel(const float *Y, const float *T, int B, int n, float *dY,
                                                        uint16_t *dYb, float *row_sq) {
  const int b = blockIdx.x;
  __shared__ float part[256];
  float s = 0.0f;
  const float scale = 2.0f / ((float)B * (float)n);
  for (int j = threadIdx.x; j < n; j += 256) {
    const int64_t o = (int64_t)b * n + j;
    const float d = Y[o] - T[o];
    s = fmaf(d, d, s);
    const float g = scale * d;
    dY[o] = g;
    dYb[o] = bf16_bits(g);
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {               // fixed pairwise tree
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) row_sq[b] = part[0];
}

// loss = sum of the row sums / (B n_out), in row order.
__global__ void loss_total_kernel(const float *row_sq, int B, int n, float *loss) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += (double)row_sq[b];
    loss[0] = (float)(s / ((double)B * (double)n));
  }
}

// dZ = dH * gelu'(Z) (float32 and bfloat16).
__global__ __launch_bounds__(256) void gelu_back_kernel(const float *dH, const float *Z, float *dZ, uint16_t *dZb,
                                                        int64_t n) {
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float d = dH[i] * gelu_grad(Z[i]);
    dZ[i] = d;
    dZb[i] = bf16_bits(d);
  }
}

// db[j] = sum over rows b of dZ[b][j], rows in order.
__global__ __launch_bounds__(256) void col_sum_kernel(const float *dZ, int B, int n, float *db) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j < n) {
    float s = 0.0f;
    for (int b = 0; b < B; ++b) s += dZ[(int64_t)b * n + j];
    db[j] = s;
  }
}

// Adam with bias correction; refreshes the bfloat16 copy of the parameters.
__global__ __launch_bounds__(256) void adam_kernel(float *theta, float *m, float *v, const float *grad,
                                                   uint16_t *theta_b, int64_t n, float lr, float b1, float b2,
                                                   float eps, float c1, float c2) {
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float t = theta[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    theta[i] = t;
    if (theta_b) theta_b[i] = bf16_bits(t);
  }
}

// Fixed-order sum of one value per thread of a 256-thread workgroup
// (butterfly within each wavefront, then the four wavefronts in order).
__device__ __forceinline__ float block_sum(float s, float *sh) {
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  const float t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return t;
}

// y[r] = alpha sum_j A[r][j] x[j] + beta y[r]: one workgroup per row, threads
// stride the row, two accumulators, fixed-order block sum.
__global__ __launch_bounds__(256) void gemv_f32_kernel(const float *A, int64_t lda, const float *x, int rows,
                                                       int cols, float alpha, float beta, float *y) {
  __shared__ float sh[4];
  const int r = blockIdx.x;
  const float *row = A + (int64_t)r * lda;
  float a0 = 0.f, a1 = 0.f;
  int j = threadIdx.x;
  for (; j + 256 < cols; j += 512) {
    a0 = fmaf(row[j], x[j], a0);
    a1 = fmaf(row[j + 256], x[j + 256], a1);
  }
  if (j < cols) a0 = fmaf(row[j], x[j], a0);
  const float s = block_sum(a0 + a1, sh);
  if (threadIdx.x == 0) y[r] = alpha * s + (beta == 0.0f ? 0.0f : beta * y[r]);
}

// Batch-1 layer of the network: z[r] = sum_k bf16(x[k]) W[r][k] + b[r] with
// bfloat16 weights and float32 accumulation (the rounding points of the
// training products); out_f32 = GELU(z) or z, out_bf16 its bfloat16 rounding.
__global__ __launch_bounds__(256) void gemv_bf16_kernel(const uint16_t *W, const float *x, const float *b, int rows,
                                                        int cols, int gelu_on, float *out_f32, uint16_t *out_bf16) {
  __shared__ float sh[4];
  const int r = blockIdx.x;
  const uint16_t *row = W + (int64_t)r * cols;
  float a0 = 0.f;
  for (int j = threadIdx.x; j < cols; j += 256)
    a0 = fmaf(__uint_as_float((uint32_t)row[j] << 16), __uint_as_float((uint32_t)bf16_bits(x[j]) << 16), a0);
  const float s = block_sum(a0, sh);
  if (threadIdx.x == 0) {
    const float z = s + (b ? b[r] : 0.0f);
    const float y = gelu_on ? gelu(z) : z;
    if (out_f32) out_f32[r] = y;
    if (out_bf16) out_bf16[r] = bf16_bits(y);
  }
}

// Predictor history: with a previous frame (push != 0), shift the window by
// one frame and append the normalised change (m - m_prev - mean) / std; then
// m_prev = m.
__global__ __launch_bounds__(256) void history_push_kernel(float *hist, int history, int n_modes, const float *m,
                                                           float *m_prev, const float *mean, const float *inv_std,
                                                           int push) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j < n_modes) {
    if (push) {
      for (int h = 0; h + 1 < history; ++h) hist[(int64_t)h * n_modes + j] = hist[(int64_t)(h + 1) * n_modes + j];
      hist[(int64_t)(history - 1) * n_modes + j] = (m[j] - m_prev[j] - mean[j]) * inv_std[j];
    }
    m_prev[j] = m[j];
  }
}

// Forecast change in physical units: d = y * std + mean (0 without a
// forecast, y == nullptr) and the forecast modes m_last + d.
__global__ __launch_bounds__(256) void denorm_kernel(const float *y, const float *m_last, const float *mean,
                                                     const float *std_, int n_modes, float *d, float *mhat) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j < n_modes) {
    const float dj = y ? fmaf(y[j], std_[j], mean[j]) : 0.0f;
    d[j] = dj;
    mhat[j] = m_last[j] + dj;
  }
}


}  // namespace

hipError_t launch_gemm(const GemmArgs &g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (g.K < 0) return hipErrorInvalidValue;
  const dim3 grid((g.N + kTile - 1) / kTile, (g.M + kTile - 1) / kTile);
  gemm_bf16_kernel<<<grid, 256, 0, st>>>(g);
  return hipGetLastError();
}

static unsigned grid_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

hipError_t launch_round_bf16(const float *x, uint16_t *y, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  round_bf16_kernel<<<grid_for(n), 256, 0, st>>>(x, y, n);
  return hipGetLastError();
}

hipError_t launch_loss_grad(const float *Y, const float *T, int B, int n, float *dY, uint16_t *dYb, float *row_sq,
                            float *loss, hipStream_t st) {
  loss_grad_kernel<<<B, 256, 0, st>>>(Y, T, B, n, dY, dYb, row_sq);
  loss_total_kernel<<<1, 64, 0, st>>>(row_sq, B, n, loss);
  return hipGetLastError();
}

hipError_t launch_gelu_back(const float *dH, const float *Z, float *dZ, uint16_t *dZb, int64_t n, hipStream_t st) {
  gelu_back_kernel<<<grid_for(n), 256, 0, st>>>(dH, Z, dZ, dZb, n);
  return hipGetLastError();
}

hipError_t launch_col_sum(const float *dZ, int B, int n, float *db, hipStream_t st) {
  col_sum_kernel<<<(n + 255) / 256, 256, 0, st>>>(dZ, B, n, db);
  return hipGetLastError();
}

hipError_t launch_adam(float *theta, float *m, float *v, const float *grad, uint16_t *theta_b, int64_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2, hipStream_t st) {
  adam_kernel<<<grid_for(n), 256, 0, st>>>(theta, m, v, grad, theta_b, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_gemv_f32(const float *A, int64_t lda, const float *x, int rows, int cols, float alpha, float beta,
                           float *y, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  gemv_f32_kernel<<<rows, 256, 0, st>>>(A, lda, x, rows, cols, alpha, beta, y);
  return hipGetLastError();
}

hipError_t launch_gemv_bf16(const uint16_t *W, const float *x, const float *b, int rows, int cols, int gelu_on,
                            float *out_f32, uint16_t *out_bf16, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  gemv_bf16_kernel<<<rows, 256, 0, st>>>(W, x, b, rows, cols, gelu_on, out_f32, out_bf16);
  return hipGetLastError();
}

hipError_t launch_history_push(float *hist, int history, int n_modes, const float *m, float *m_prev,
                               const float *mean, const float *inv_std, int push, hipStream_t st) {
  history_push_kernel<<<(n_modes + 255) / 256, 256, 0, st>>>(hist, history, n_modes, m, m_prev, mean, inv_std,
                                                              push);
  return hipGetLastError();
}

hipError_t launch_denorm(const float *y, const float *m_last, const float *mean, const float *std_, int n_modes,
                         float *d, float *mhat, hipStream_t st) {
  denorm_kernel<<<(n_modes + 255) / 256, 256, 0, st>>>(y, m_last, mean, std_, n_modes, d, mhat);
  return hipGetLastError();
}


}  // namespace rtcm
