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
//   pred_*_kernel      the predictor step in four launches: modes and their
//                      history, network layer 1, layer 2 with the forecast,
//                      feed-forward slopes
//
// Every reduction has a fixed order: results are run-to-run deterministic.
#include "mlp_kernels.h"
#include "pred_device.h"

#include <algorithm>
#include <climits>

namespace rtcm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float gelu_grad(float z) {
  const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * z * z);
  return cdf + z * pdf;
}

// ---------------------------------------------------------------------------
// GEMM.  Workgroup = 4 wavefronts computing a BM x BN tile of C (64 x 64);
// wavefront w owns rows [(w / 2) BM / 2, +BM / 2) and columns
// [(w % 2) BN / 2, +BN / 2), that is (BM / 64) x (BN / 64) blocks of 32 x 32.  K is walked in tiles
// of 64 through two LDS buffers: the next tile is loaded into registers while
// the matrix cores work on the current one.  A tile is read in runs of 4
// elements along the operand's contiguous dimension (k for X W^T, m or n for
// the weight gradients), one 8- or 16-byte load per run where the rows are
// aligned, element by element otherwise.  The K range may be split over
// `splits` workgroups whose float32 partial tiles a second kernel adds in
// split order.
// Tile order: the grid is one-dimensional and workgroup L runs on XCD L mod 8
// (the dispatcher deals workgroups to the eight XCDs in turn), so XCD x takes
// the contiguous range [x per, (x + 1) per) of a logical order in which the
// split is slowest and, within a split, the tiles that share the smaller
// operand's panels are adjacent (M tiles fastest when A is the smaller
// operand): each XCD's L2 then holds the panels its workgroups read instead of
// every XCD streaming both operands whole.
// Operand layout of the 32x32x16 operation: lane l supplies row (A) or column
// (B) l % 32 and the eight consecutive k = 8 (l / 32) .. 8 (l / 32) + 7; its
// 16 results are column l % 32, rows 8 (v / 4) + 4 (l / 32) + v % 4.
constexpr int kKT = 64, kKP = kKT + 8;

__device__ __forceinline__ void gemm_epilogue(const GemmArgs &g, int m, int n, float acc) {
  float z = g.alpha * acc;
  if (g.bias) z += g.bias[n];
  const int64_t o = (int64_t)m * g.ldc + n;
  if (g.c_pre) g.c_pre[o] = z;
  const float y = g.gelu ? gelu(z) : z;
  if (g.c_f32) g.c_f32[o] = y;
  if (g.c_bf16) g.c_bf16[o] = bf16_bits(y);
}

// One operand of a tile: R rows (m of A or n of B) x kKT k.  Element (i, k) of
// the operand matrix is at f32 / b16 + i si + k sk; `kc`: contiguous along k
// (sk == 1) else along i (si == 1); `vec`: runs of 4 may be read as one load.
struct Operand {
  const float *f32;
  const uint16_t *b16;
  int64_t si, sk;
  int rows;                                        // valid i (M or N)
  bool kc, vec;
};

template <int R>
struct TileRegs {
  static constexpr int NV = R * kKT / 4 / 256;     // runs of 4 per thread
  uint2 v[NV];                                     // 4 bfloat16 codes of a run, packed
};

__device__ __forceinline__ uint2 pack4(uint16_t a, uint16_t b, uint16_t c, uint16_t d) {
  return make_uint2((uint32_t)a | ((uint32_t)b << 16), (uint32_t)c | ((uint32_t)d << 16));
}
__device__ __forceinline__ uint16_t unpack4(const uint2 &x, int e) {
  const uint32_t w = e < 2 ? x.x : x.y;
  return (uint16_t)((e & 1) ? (w >> 16) : (w & 0xffffu));
}

// Run r of this thread: first element (i, kk) and direction.
template <int R>
__device__ __forceinline__ void run_pos(const Operand &o, int r, int &i, int &kk) {
  const int q = r * 256 + threadIdx.x;
  if (o.kc) {
    i = q / (kKT / 4);
    kk = (q % (kKT / 4)) * 4;
  } else {
    kk = q / (R / 4);
    i = (q % (R / 4)) * 4;
  }
}

// Any strides: a run is read with one load where it is aligned (o.vec) and
// whole, element by element otherwise.
template <int R>
__device__ __forceinline__ void load_tile(const Operand &o, int i0, int k0, int k_end, TileRegs<R> &t) {
#pragma unroll
  for (int r = 0; r < TileRegs<R>::NV; ++r) {
    int i, kk;
    run_pos<R>(o, r, i, kk);
    const int gi = i0 + i, gk = k0 + kk;
    const int64_t base = (int64_t)gi * o.si + (int64_t)gk * o.sk;
    const bool whole = o.kc ? (gi < o.rows && gk + 3 < k_end) : (gi + 3 < o.rows && gk < k_end);
    if (o.vec && whole) {
      if (o.f32) {
        const float4 x = *reinterpret_cast<const float4 *>(o.f32 + base);
        t.v[r] = pack4(bf16_bits(x.x), bf16_bits(x.y), bf16_bits(x.z), bf16_bits(x.w));
      } else {
        t.v[r] = *reinterpret_cast<const uint2 *>(o.b16 + base);
      }
    } else {
      uint16_t x[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int ei = gi + (o.kc ? 0 : e), ek = gk + (o.kc ? e : 0);
        x[e] = 0;
        if (ei < o.rows && ek < k_end) {
          const int64_t off = (int64_t)ei * o.si + (int64_t)ek * o.sk;
          x[e] = o.f32 ? bf16_bits(o.f32[off]) : o.b16[off];
        }
      }
      t.v[r] = pack4(x[0], x[1], x[2], x[3]);
    }
  }
}

template <int R>
__device__ __forceinline__ void store_tile(const Operand &o, const TileRegs<R> &t, uint16_t (*S)[kKP]) {
#pragma unroll
  for (int r = 0; r < TileRegs<R>::NV; ++r) {
    int i, kk;
    run_pos<R>(o, r, i, kk);
    if (o.kc) {
      *reinterpret_cast<uint2 *>(&S[i][kk]) = t.v[r];
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) S[i + e][kk] = unpack4(t.v[r], e);
    }
  }
}

// Aligned operands (VEC) with their contiguous dimension fixed at compile time
// (KC: along k): a thread's runs keep their rows for the whole K range, so
// their offsets are computed once and a tile's loads add only the uniform
// offset of its first k.
template <int R, bool KC>
struct RunAddr {
  static constexpr int NV = TileRegs<R>::NV;
  int64_t off[NV];           // element offset of run r at k = 0
  int kk[NV];                // k of run r within a tile
  bool rows_ok[NV];          // run r's rows lie inside the matrix
};

// Operands contiguous along i (not KC): a thread's runs form a 4 x NV block,
// rows i..i+3 of the run at k = NV (t / (R / 4)) + r, so that store_tile_vec
// can transpose the block in registers and store whole k-runs.
template <int R, bool KC>
__device__ __forceinline__ void run_addr(const Operand &o, int i0, RunAddr<R, KC> &a) {
  constexpr int NV = RunAddr<R, KC>::NV;
  static_assert(KC || NV % 4 == 0, "k-runs of 4 per block");
#pragma unroll
  for (int r = 0; r < NV; ++r) {
    const int q = r * 256 + threadIdx.x;
    const int i = KC ? q / (kKT / 4) : ((int)threadIdx.x % (R / 4)) * 4;
    const int kk = KC ? (q % (kKT / 4)) * 4 : NV * ((int)threadIdx.x / (R / 4)) + r;
    const int gi = i0 + i;
    a.off[r] = (int64_t)gi * o.si + (int64_t)kk * o.sk;
    a.kk[r] = kk;
    a.rows_ok[r] = KC ? gi < o.rows : gi + 3 < o.rows;
  }
}

// F32: the operand is float32 (rounded to bfloat16 as read), else bfloat16.
template <int R, bool KC, bool F32>
__device__ __forceinline__ void load_tile_vec(const Operand &o, const RunAddr<R, KC> &a, int k0, int k_end,
                                              TileRegs<R> &t) {
  const int64_t koff = (int64_t)k0 * o.sk;
#pragma unroll
  for (int r = 0; r < RunAddr<R, KC>::NV; ++r) {
    const bool whole = a.rows_ok[r] && (KC ? k0 + a.kk[r] + 3 < k_end : k0 + a.kk[r] < k_end);
    uint2 x = make_uint2(0u, 0u);
    if (whole) {
      const int64_t e = a.off[r] + koff;
      if constexpr (F32) {
        const float4 y = *reinterpret_cast<const float4 *>(o.f32 + e);
        x = pack4(bf16_bits(y.x), bf16_bits(y.y), bf16_bits(y.z), bf16_bits(y.w));
      } else {
        x = *reinterpret_cast<const uint2 *>(o.b16 + e);
      }
    }
    t.v[r] = x;
  }
}

template <int R, bool KC>
__device__ __forceinline__ void store_tile_vec(const TileRegs<R> &t, uint16_t (*S)[kKP]) {
  constexpr int NV = TileRegs<R>::NV;
  if constexpr (KC) {
#pragma unroll
    for (int r = 0; r < NV; ++r) {
      const int q = r * 256 + threadIdx.x;
      *reinterpret_cast<uint2 *>(&S[q / (kKT / 4)][(q % (kKT / 4)) * 4]) = t.v[r];
    }
  } else {
    // the thread's 4 x NV block (rows i..i+3, k = k0..k0+NV-1), transposed in
    // registers four k at a time: row i+e gets (v[r].e, v[r+1].e, v[r+2].e, v[r+3].e)
    const int i = ((int)threadIdx.x % (R / 4)) * 4, k0 = NV * ((int)threadIdx.x / (R / 4));
#pragma unroll
    for (int r = 0; r < NV; r += 4) {
      const uint2 a = t.v[r], b = t.v[r + 1], c = t.v[r + 2], d = t.v[r + 3];
      const uint32_t lo = 0xffffu, hi = 0xffff0000u;
      *reinterpret_cast<uint2 *>(&S[i + 0][k0 + r]) =
          make_uint2((a.x & lo) | (b.x << 16), (c.x & lo) | (d.x << 16));
      *reinterpret_cast<uint2 *>(&S[i + 1][k0 + r]) =
          make_uint2((a.x >> 16) | (b.x & hi), (c.x >> 16) | (d.x & hi));
      *reinterpret_cast<uint2 *>(&S[i + 2][k0 + r]) =
          make_uint2((a.y & lo) | (b.y << 16), (c.y & lo) | (d.y << 16));
      *reinterpret_cast<uint2 *>(&S[i + 3][k0 + r]) =
          make_uint2((a.y >> 16) | (b.y & hi), (c.y >> 16) | (d.y & hi));
    }
  }
}

struct GemmTiles {
  int ntm, ntn, splits;      // M tiles, N tiles, K splits
  int per;                   // logical tiles per XCD
  int m_fast;                // M tiles vary fastest within a split
};

// VEC: both operands aligned (runs of 4 read whole), with A contiguous along k
// when KA and B when KB, A float32 when AF (B bfloat16); otherwise (not VEC)
// any strides and types, read element-wise where a run is not whole.
template <int BM, int BN, bool VEC, bool KA, bool KB, bool AF>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g, int k_chunk, int a_vec, int b_vec, GemmTiles tl) {
  constexpr int MB = BM / 64, NB = BN / 64;        // 32 x 32 blocks per wavefront along m and n
  __shared__ __align__(16) uint16_t As[2][BM][kKP];   // [m][k]
  __shared__ __align__(16) uint16_t Bs[2][BN][kKP];   // [n][k]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int per_split = tl.ntm * tl.ntn;
  const int lt = (int)(blockIdx.x % 8u) * tl.per + (int)(blockIdx.x / 8u);   // logical tile
  if (lt >= per_split * tl.splits) return;        // the grid is rounded up to 8 XCD ranges
  const int kz = lt / per_split, rt = lt - kz * per_split;
  const int tm = tl.m_fast ? rt % tl.ntm : rt / tl.ntn;
  const int tn = tl.m_fast ? rt / tl.ntm : rt % tl.ntn;
  const int m0 = tm * BM, n0 = tn * BN;
  const int kb0 = kz * k_chunk;
  const int kb1 = min(g.K, kb0 + k_chunk);
  const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);
  const Operand A{g.a_f32, g.a_bf16, g.sam, g.sak, g.M, g.sak == 1, a_vec != 0};
  const Operand B{g.b_f32, g.b_bf16, g.sbn, g.sbk, g.N, g.sbk == 1, b_vec != 0};
  f32x16 acc[MB][NB];
#pragma unroll
  for (int b = 0; b < MB; ++b)
#pragma unroll
    for (int c = 0; c < NB; ++c)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[b][c][v] = 0.0f;

  TileRegs<BM> ra;
  TileRegs<BN> rb;
  [[maybe_unused]] RunAddr<BM, KA> aa;
  [[maybe_unused]] RunAddr<BN, KB> ab;
  if constexpr (VEC) {
    run_addr<BM, KA>(A, m0, aa);
    run_addr<BN, KB>(B, n0, ab);
  }
  auto load = [&](int k0) {
    if constexpr (VEC) {
      load_tile_vec<BM, KA, AF>(A, aa, k0, kb1, ra);
      load_tile_vec<BN, KB, false>(B, ab, k0, kb1, rb);
    } else {
      load_tile<BM>(A, m0, k0, kb1, ra);
      load_tile<BN>(B, n0, k0, kb1, rb);
    }
  };
  auto store = [&](int buf) {
    if constexpr (VEC) {
      store_tile_vec<BM, KA>(ra, As[buf]);
      store_tile_vec<BN, KB>(rb, Bs[buf]);
    } else {
      store_tile<BM>(A, ra, As[buf]);
      store_tile<BN>(B, rb, Bs[buf]);
    }
  };
  if (kb0 < kb1) {
    load(kb0);
    store(0);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = kb0; k0 < kb1; k0 += kKT) {
    const bool more = k0 + kKT < kb1;
    if (more) load(k0 + kKT);                       // in flight while the matrix cores work
#pragma unroll
    for (int ks = 0; ks < kKT; ks += 16) {
      const int kq = ks + 8 * (lane >> 5);
      bf16x8 bv[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c)
        bv[c] = *reinterpret_cast<const bf16x8 *>(&Bs[buf][wn + 32 * c + (lane & 31)][kq]);
#pragma unroll
      for (int b = 0; b < MB; ++b) {
        const bf16x8 av = *reinterpret_cast<const bf16x8 *>(&As[buf][wm + 32 * b + (lane & 31)][kq]);
#pragma unroll
        for (int c = 0; c < NB; ++c) acc[b][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv[c], acc[b][c], 0, 0, 0);
      }
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

#pragma unroll
  for (int c = 0; c < NB; ++c) {
    const int n = n0 + wn + 32 * c + (lane & 31);
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int m = m0 + wm + 32 * b + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        if (m < g.M && n < g.N) {
          if (tl.splits == 1) gemm_epilogue(g, m, n, acc[b][c][v]);
          else g.ws[((int64_t)kz * g.M + m) * g.N + n] = acc[b][c][v];
        }
      }
  }
}

// Sum of the split-K partial tiles in split order, then the epilogue.
__global__ __launch_bounds__(256) void gemm_split_sum_kernel(GemmArgs g, int splits) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t mn = (int64_t)g.M * g.N;
  if (t >= mn) return;
  float s = g.ws[t];
  for (int z = 1; z < splits; ++z) s += g.ws[(int64_t)z * mn + t];
  gemm_epilogue(g, (int)(t / g.N), (int)(t % g.N), s);
}

// ---------------------------------------------------------------------------
// elementwise and reductions
__global__ __launch_bounds__(256) void round_bf16_kernel(const float *x, uint16_t *y, int64_t n) {
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) y[i] = bf16_bits(x[i]);
}

// dY = 2 (Y - T) / (B n_out) (float32 and bfloat16) and per-row sums of (Y - T)^2.
__device__ __forceinline__ float split_sum(const float *parts, int splits, int64_t mn, int64_t o) {
  float s = parts[o];
  for (int z = 1; z < splits; ++z) s += parts[(int64_t)z * mn + o];
  return s;
}

__global__ __launch_bounds__(256) void loss_grad_kernel(const float *Y, const float *T, int B, int n, float *dY,
                                                        uint16_t *dYb, float *row_sq, const float *parts, int splits,
                                                        const float *bias) {
  const int b = blockIdx.x;
  __shared__ float part[256];
  float s = 0.0f;
  const float scale = 2.0f / ((float)B * (float)n);
  for (int j = threadIdx.x; j < n; j += 256) {
    const int64_t o = (int64_t)b * n + j;
    float y;
    if (splits > 0) {                               // the product's epilogue: 1 * sum + bias
      y = split_sum(parts, splits, (int64_t)B * n, o);
      if (bias) y += bias[j];
    } else {
      y = Y[o];
    }
    const float d = y - T[o];
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
// loss = sum of the row sums (float64; thread t adds rows t, t + 256, ... in
// order, then a fixed pairwise tree) / (B n).
__global__ __launch_bounds__(256) void loss_total_kernel(const float *row_sq, int B, int n, float *loss) {
  __shared__ double part[256];
  double s = 0.0;
  for (int b = threadIdx.x; b < B; b += 256) s += (double)row_sq[b];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = (float)(part[0] / ((double)B * (double)n));
}

// dZ = dH * gelu'(Z) (float32 and bfloat16).
__global__ __launch_bounds__(256) void gelu_back_kernel(const float *dH, const float *Z, float *dZ, uint16_t *dZb,
                                                        int64_t n, const float *parts, int splits) {
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float h = splits > 0 ? split_sum(parts, splits, n, i) : dH[i];
    const float d = h * gelu_grad(Z[i]);
    dZ[i] = d;
    dZb[i] = bf16_bits(d);
  }
}

// db[j] = sum over rows b of dZ[b][j]: a workgroup of 16 wavefronts takes 64
// columns; wavefront r adds rows r, r + 16, ... in order (8 loads in flight),
// then the 16 partial sums are added in a fixed pairwise tree.
__global__ __launch_bounds__(1024) void col_sum_kernel(const float *dZ, int B, int n, float *db) {
  __shared__ float part[16][64];
  const int c = threadIdx.x & 63, r = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + c;
  float s = 0.0f;
  if (j < n) {
    int b = r;
    for (; b + 16 * 7 < B; b += 16 * 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = dZ[(int64_t)(b + 16 * u) * n + j];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; b < B; b += 16) s += dZ[(int64_t)b * n + j];
  }
  part[r][c] = s;
  __syncthreads();
  for (int w = 8; w > 0; w >>= 1) {
    if (r < w) part[r][c] += part[r + w][c];
    __syncthreads();
  }
  if (r == 0 && j < n) db[j] = part[0][c];
}

// Adam with bias correction on element i; refreshes the bfloat16 copy of the parameters.
__device__ __forceinline__ void adam_element(const AdamTensor &t, int64_t i, float lr, float b1, float b2, float eps,
                                             float c1, float c2) {
  const float g = t.grad[i];
  const float mi = b1 * t.m[i] + (1.0f - b1) * g;
  const float vi = b2 * t.v[i] + (1.0f - b2) * g * g;
  t.m[i] = mi;
  t.v[i] = vi;
  const float th = t.theta[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  t.theta[i] = th;
  if (t.theta_b) t.theta_b[i] = bf16_bits(th);
}

// Adam on several tensors in one launch: workgroups [first[k], first[k + 1]) take
// tensor k, kAdamChunk consecutive elements each (the choice of tensor is
// uniform per workgroup).
constexpr int kAdamChunk = 1024;
struct AdamSet {
  AdamTensor t[kAdamTensors];
  int32_t first[kAdamTensors + 1];
  int32_t count;
};

__global__ __launch_bounds__(256) void adam_multi_kernel(AdamSet s, float lr, float b1, float b2, float eps, float c1,
                                                         float c2) {
  const int32_t w = (int32_t)blockIdx.x;
  AdamTensor t = s.t[0];
  int32_t w0 = 0;
#pragma unroll
  for (int k = 1; k < kAdamTensors; ++k)
    if (k < s.count && w >= s.first[k]) {
      t = s.t[k];
      w0 = s.first[k];
    }
  const int64_t e0 = (int64_t)(w - w0) * kAdamChunk;
  for (int64_t i = e0 + threadIdx.x; i < t.n && i < e0 + kAdamChunk; i += 256)
    adam_element(t, i, lr, b1, b2, eps, c1, c2);
}

// The predictor step's four launches (arithmetic in pred_device.h): one
// workgroup per mode, per hidden unit and per mode, then one wavefront per
// slope.
__global__ __launch_bounds__(256) void pred_modes_kernel(PredStepArgs a) {
  __shared__ float sh[8];
  pred_modes<1, false>(a, blockIdx.x, 1, 1, a.push != 0, a.pos, VecPlain{a.s}, VecPlain{a.c}, sh);
}

template <bool VEC>
__global__ __launch_bounds__(256) void pred_hidden_kernel(PredStepArgs a) {
  __shared__ float sh[4];
  pred_hidden<VEC, 1, false>(a, blockIdx.x, 1, 1, VecPlain{a.hist + (int64_t)(a.pos + 1) * a.n_modes}, sh);
}

template <bool VEC>
__global__ __launch_bounds__(256) void pred_forecast_kernel(PredStepArgs a) {
  __shared__ float sh[4];
  pred_forecast<VEC, 1, false>(a, blockIdx.x, 1, 1, a.full != 0, VecPlain{a.h}, sh);
}

__global__ __launch_bounds__(256) void pred_slopes_kernel(PredStepArgs a) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= a.n_slopes) return;
  float v[1];
  pred_slopes<1>(a, i, 1, 1, lane, VecPlain{a.d}, VecPlain{a.s}, v);
  if (lane == 0) a.s_out[i] = v[0];
}

}  // namespace

hipError_t launch_gemm(const GemmArgs &g, hipStream_t st, int *deferred) {
  if (deferred) *deferred = 0;
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (g.K < 0) return hipErrorInvalidValue;
  // 64 x 64 tiles; the K range is split until about 512 workgroups run (two
  // per compute unit), within the workspace
  // the aligned-run kernels need every run wholly inside or outside the matrix
  auto vec_ok = [](const void *p, int bytes, int64_t s_run, int64_t s_other) {
    return s_run == 1 && s_other % 4 == 0 && (reinterpret_cast<uintptr_t>(p) % (4 * bytes)) == 0;
  };
  const void *pa = g.a_f32 ? (const void *)g.a_f32 : (const void *)g.a_bf16;
  const void *pb = g.b_f32 ? (const void *)g.b_f32 : (const void *)g.b_bf16;
  const int ab = g.a_f32 ? 4 : 2, bb = g.b_f32 ? 4 : 2;
  const int a_vec = g.sak == 1 ? vec_ok(pa, ab, g.sak, g.sam) : vec_ok(pa, ab, g.sam, g.sak);
  const int b_vec = g.sbk == 1 ? vec_ok(pb, bb, g.sbk, g.sbn) : vec_ok(pb, bb, g.sbn, g.sbk);
  const bool all_vec = a_vec && b_vec && g.M % 4 == 0 && g.N % 4 == 0 && g.K % 4 == 0;
  // (128 x 128 tiles measured slower at these sizes: the K range per workgroup
  // is a few tiles, so the pipeline's start and end dominate)
  constexpr int bm = 64, bn = 64;
  const int tiles = ((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn);
  const int k_tiles = (g.K + kKT - 1) / kKT;
  const int target = 512;
  int splits = (target + tiles - 1) / tiles;
  splits = std::min(splits, std::max(1, k_tiles / 2));
  if (g.ws == nullptr) splits = 1;
  else splits = (int)std::min<int64_t>(splits, g.ws_len / ((int64_t)g.M * g.N));
  if (splits < 1) splits = 1;
  const int k_chunk = ((k_tiles + splits - 1) / splits) * kKT;
  splits = std::max(1, (g.K + k_chunk - 1) / k_chunk);
  GemmTiles tl{};
  tl.ntm = (g.M + bm - 1) / bm;
  tl.ntn = (g.N + bn - 1) / bn;
  tl.splits = splits;
  const int64_t total = (int64_t)tl.ntm * tl.ntn * splits;
  tl.per = (int)((total + 7) / 8);
  // the operand whose panels every XCD reads whole is the smaller one
  const int64_t a_bytes = (int64_t)g.M * g.K * ab, b_bytes = (int64_t)g.N * g.K * bb;
  tl.m_fast = a_bytes <= b_bytes ? 1 : 0;
  const dim3 grid((unsigned)(8 * tl.per));
  if (all_vec && g.b_f32 == nullptr) {
    const bool ka = g.sak == 1, kb = g.sbk == 1, af = g.a_f32 != nullptr;
    auto go = [&](auto kern) { kern<<<grid, 256, 0, st>>>(g, k_chunk, a_vec, b_vec, tl); };
    if (af) {
      if (ka && kb) go(gemm_bf16_kernel<64, 64, true, true, true, true>);
      else if (ka) go(gemm_bf16_kernel<64, 64, true, true, false, true>);
      else if (kb) go(gemm_bf16_kernel<64, 64, true, false, true, true>);
      else go(gemm_bf16_kernel<64, 64, true, false, false, true>);
    } else {
      if (ka && kb) go(gemm_bf16_kernel<64, 64, true, true, true, false>);
      else if (ka) go(gemm_bf16_kernel<64, 64, true, true, false, false>);
      else if (kb) go(gemm_bf16_kernel<64, 64, true, false, true, false>);
      else go(gemm_bf16_kernel<64, 64, true, false, false, false>);
    }
  } else {
    gemm_bf16_kernel<64, 64, false, false, false, false><<<grid, 256, 0, st>>>(g, k_chunk, a_vec, b_vec, tl);
  }
  if (splits > 1 && deferred && g.alpha == 1.0f && !g.gelu) {
    *deferred = splits;                             // the consumer adds the partials
    return hipGetLastError();
  }
  if (splits > 1) {
    const int64_t mn = (int64_t)g.M * g.N;
    gemm_split_sum_kernel<<<(unsigned)((mn + 255) / 256), 256, 0, st>>>(g, splits);
  }
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
                            float *loss, hipStream_t st, const float *parts, int splits, const float *bias) {
  loss_grad_kernel<<<B, 256, 0, st>>>(Y, T, B, n, dY, dYb, row_sq, parts, splits, bias);
  loss_total_kernel<<<1, 256, 0, st>>>(row_sq, B, n, loss);
  return hipGetLastError();
}

hipError_t launch_gelu_back(const float *dH, const float *Z, float *dZ, uint16_t *dZb, int64_t n, hipStream_t st,
                            const float *parts, int splits) {
  gelu_back_kernel<<<grid_for(n), 256, 0, st>>>(dH, Z, dZ, dZb, n, parts, splits);
  return hipGetLastError();
}

hipError_t launch_col_sum(const float *dZ, int B, int n, float *db, hipStream_t st) {
  col_sum_kernel<<<(n + 63) / 64, 1024, 0, st>>>(dZ, B, n, db);
  return hipGetLastError();
}

hipError_t launch_adam_multi(const AdamTensor *t, int count, float lr, float b1, float b2, float eps, float c1,
                             float c2, hipStream_t st) {
  if (count < 1 || count > kAdamTensors) return hipErrorInvalidValue;
  AdamSet s{};
  int64_t blocks = 0;
  for (int k = 0; k < count; ++k) {
    if (t[k].n < 0) return hipErrorInvalidValue;
    s.t[k] = t[k];
    s.first[k] = (int32_t)blocks;
    blocks += (t[k].n + kAdamChunk - 1) / kAdamChunk;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
  }
  s.first[count] = (int32_t)blocks;
  s.count = count;
  if (blocks == 0) return hipSuccess;
  adam_multi_kernel<<<(unsigned)blocks, 256, 0, st>>>(s, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_pred_step(const PredStepArgs &a, hipStream_t st) {
  if (a.n_modes <= 0 || a.n_slopes <= 0) return hipErrorInvalidValue;
  pred_modes_kernel<<<a.n_modes, 256, 0, st>>>(a);
  hipError_t e = hipGetLastError();
  // 8-byte weight loads when every row starts 8-byte aligned
  const bool v1 = a.n_in % 4 == 0 && reinterpret_cast<uintptr_t>(a.W1) % 8 == 0;
  const bool v2 = a.n_hid % 4 == 0 && reinterpret_cast<uintptr_t>(a.W2) % 8 == 0;
  if (e == hipSuccess && a.full) {
    if (v1)
      pred_hidden_kernel<true><<<a.n_hid, 256, 0, st>>>(a);
    else
      pred_hidden_kernel<false><<<a.n_hid, 256, 0, st>>>(a);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    if (v2)
      pred_forecast_kernel<true><<<a.n_modes, 256, 0, st>>>(a);
    else
      pred_forecast_kernel<false><<<a.n_modes, 256, 0, st>>>(a);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    pred_slopes_kernel<<<(a.n_slopes + 3) / 4, 256, 0, st>>>(a);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace rtcm
