// Device arithmetic of one step of the learned predictor, shared by the
// predictor's own four launches and by the predictive persistent frames.
// Every vector an operation reads goes through an accessor (plain loads, or
// device-coherent loads of values other workgroups of the same launch wrote),
// and every value a later phase reads elsewhere is stored plainly or
// device-coherently (COH): the accessors change the loads, never the
// arithmetic or its order, so both forms give the same bits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pred_step.h"

namespace rtcm {

// bfloat16 of a float, round to nearest even (NaN stays a quiet NaN).
__device__ __forceinline__ uint16_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_value(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ float bf16_round(float x) { return bf16_value(bf16_bits(x)); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

// Vector accessors.
struct VecPlain {
  const float *x;
  __device__ __forceinline__ float operator()(int64_t k) const { return x[k]; }
};
struct VecCoh {
  const float *x;
  __device__ __forceinline__ float operator()(int64_t k) const {
    return __hip_atomic_load(x + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
};

template <bool COH>
__device__ __forceinline__ void put(float *p, float v) {
  if constexpr (COH)
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    *p = v;
}

__device__ __forceinline__ float wave_total(float t) {
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
  return t;
}

// Fixed-order sums of two values per thread of a 256-thread workgroup
// (butterflies within each wavefront, then the four wavefronts in order).
__device__ __forceinline__ float2 block_sum2(float a, float b, float *sh) {
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off);
    b += __shfl_xor(b, off);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[threadIdx.x >> 6] = a;
    sh[4 + (threadIdx.x >> 6)] = b;
  }
  __syncthreads();
  const float2 t = make_float2((sh[0] + sh[1]) + (sh[2] + sh[3]), (sh[4] + sh[5]) + (sh[6] + sh[7]));
  __syncthreads();
  return t;
}

// One thread's share of the dot products of R float32 rows (row r at row0 +
// r ld, 16-byte aligned, zero-padded to a multiple of 4 elements; rows from nr
// on repeat row nr - 1 and their sums are not used) with x[0, n), the threads
// of a group of NT taking the 4-element chunks first, first + NT, ...: per
// row one accumulator per position in the chunk, added pairwise.  The chunks
// are loaded B at a time, the x values once for all rows and every load of a
// batch issued before the first product (positions past the row repeat its
// last chunk and are masked); the one partial chunk at the end of a row is
// handled apart.  Each row's sum is the same whatever R is.
template <int NT, int B, int R, class V>
__device__ __forceinline__ void rows_part_f32(const float *row0, int64_t ld, int nr, V x, int n, int first,
                                              float (&t)[R]) {
  const int nf = n >> 2;
#pragma unroll
  for (int r = 0; r < R; ++r) t[r] = 0.f;
  for (int q0 = first; q0 < nf; q0 += B * NT) {
    float4 v[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int q = min(q0 + b * NT, nf - 1);
      v[b] = make_float4(x(4 * q), x(4 * q + 1), x(4 * q + 2), x(4 * q + 3));
    }
    float4 w[R][B];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float4 *r4 = reinterpret_cast<const float4 *>(row0 + (int64_t)min(r, nr - 1) * ld);
#pragma unroll
      for (int b = 0; b < B; ++b) w[r][b] = r4[min(q0 + b * NT, nf - 1)];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const bool ok = q0 + b * NT < nf;
        a0 = ok ? fmaf(w[r][b].x, v[b].x, a0) : a0;
        a1 = ok ? fmaf(w[r][b].y, v[b].y, a1) : a1;
        a2 = ok ? fmaf(w[r][b].z, v[b].z, a2) : a2;
        a3 = ok ? fmaf(w[r][b].w, v[b].w, a3) : a3;
      }
      t[r] += (a0 + a1) + (a2 + a3);
    }
  }
  // the partial chunk nf of a row belongs to the thread whose chunks it continues
  if ((n & 3) != 0 && first == nf % NT) {
    const int k = 4 * nf, rem = n & 3;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float4 w = reinterpret_cast<const float4 *>(row0 + (int64_t)min(r, nr - 1) * ld)[nf];
      float u = w.x * x(k);
      if (rem > 1) u = fmaf(w.y, x(k + 1), u);
      if (rem > 2) u = fmaf(w.z, x(k + 2), u);
      t[r] += u;
    }
  }
}

template <int NT, int B, class V>
__device__ __forceinline__ float row_part_f32(const float *row, V x, int n, int first) {
  float t[1];
  rows_part_f32<NT, B, 1>(row, 0, 1, x, n, first, t);
  return t[0];
}

// sum_k W[k] bf16(x[k]) over k < n for R bfloat16 rows (row r at row0 + r ld;
// rows from nr on repeat row nr - 1) by a 256-thread workgroup, float32
// accumulation.  With VEC (n a multiple of 4, rows 8-byte aligned) thread t
// takes the 4-element groups t, t + 256, ..., loaded B = 4 at a time with one
// 8-byte load each (past the row: the last group again, masked), the x values
// once for all rows, one accumulator per position; otherwise element t + 256
// i goes to accumulator i mod 4.
// Each row's four accumulators are added pairwise, then over the workgroup
// in a fixed order (butterfly within each wavefront, then the four
// wavefronts in order).  sh: 4 R floats of LDS.
template <bool VEC, int R, class V>
__device__ __forceinline__ void rows_dot_bf16(const uint16_t *row0, int64_t ld, int nr, V x, int n, float *sh,
                                              float (&out)[R]) {
  float a0[R], a1[R], a2[R], a3[R];
#pragma unroll
  for (int r = 0; r < R; ++r) a0[r] = a1[r] = a2[r] = a3[r] = 0.f;
  if constexpr (VEC) {
    constexpr int B = 4;
    const int ng = n >> 2;
    for (int q0 = threadIdx.x; q0 < ng; q0 += B * 256) {
      float4 v[B];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int q = min(q0 + b * 256, ng - 1);
        v[b] = make_float4(x(4 * q), x(4 * q + 1), x(4 * q + 2), x(4 * q + 3));
      }
      uint2 w[R][B];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint2 *r2 = reinterpret_cast<const uint2 *>(row0 + (int64_t)min(r, nr - 1) * ld);
#pragma unroll
        for (int b = 0; b < B; ++b) w[r][b] = r2[min(q0 + b * 256, ng - 1)];
      }
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int b = 0; b < B; ++b) {
          const bool ok = q0 + b * 256 < ng;
          a0[r] = ok ? fmaf(__uint_as_float(w[r][b].x << 16), bf16_round(v[b].x), a0[r]) : a0[r];
          a1[r] = ok ? fmaf(__uint_as_float(w[r][b].x & 0xffff0000u), bf16_round(v[b].y), a1[r]) : a1[r];
          a2[r] = ok ? fmaf(__uint_as_float(w[r][b].y << 16), bf16_round(v[b].z), a2[r]) : a2[r];
          a3[r] = ok ? fmaf(__uint_as_float(w[r][b].y & 0xffff0000u), bf16_round(v[b].w), a3[r]) : a3[r];
        }
    }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint16_t *row = row0 + (int64_t)min(r, nr - 1) * ld;
      int k = threadIdx.x;
      for (; k + 768 < n; k += 1024) {
        a0[r] = fmaf(bf16_value(row[k]), bf16_round(x(k)), a0[r]);
        a1[r] = fmaf(bf16_value(row[k + 256]), bf16_round(x(k + 256)), a1[r]);
        a2[r] = fmaf(bf16_value(row[k + 512]), bf16_round(x(k + 512)), a2[r]);
        a3[r] = fmaf(bf16_value(row[k + 768]), bf16_round(x(k + 768)), a3[r]);
      }
      if (k < n) a0[r] = fmaf(bf16_value(row[k]), bf16_round(x(k)), a0[r]);
      if (k + 256 < n) a1[r] = fmaf(bf16_value(row[k + 256]), bf16_round(x(k + 256)), a1[r]);
      if (k + 512 < n) a2[r] = fmaf(bf16_value(row[k + 512]), bf16_round(x(k + 512)), a2[r]);
    }
  }
  float s[R];
#pragma unroll
  for (int r = 0; r < R; ++r) s[r] = (a0[r] + a1[r]) + (a2[r] + a3[r]);
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int r = 0; r < R; ++r) s[r] += __shfl_xor(s[r], off);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int r = 0; r < R; ++r) sh[4 * r + (threadIdx.x >> 6)] = s[r];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) out[r] = (sh[4 * r] + sh[4 * r + 1]) + (sh[4 * r + 2] + sh[4 * r + 3]);
  __syncthreads();
}

template <bool VEC, class V>
__device__ __forceinline__ float row_dot_bf16(const uint16_t *row, V x, int n, float *sh) {
  float out[1];
  rows_dot_bf16<VEC, 1>(row, 0, 1, x, n, sh, out);
  return out[0];
}

// The step's rows are taken R at a time, rows j0 + r dj (r < nr) of one
// kind; the x values are then loaded once for the R rows and every row's
// loads are in flight together.  Each row's arithmetic is the same for every
// R, so the step's own launches (one row per workgroup) and the persistent
// frames (a few rows per workgroup) give the same bits.

// Step 1 for modes j = j0 + r dj, by a 256-thread workgroup: m_j = P_j s +
// (P D)_j c_prev (the two dot products reduced together); after a previous
// frame (push) the normalised change (m_j - m_prev_j - mean_j) / std_j goes
// to ring slots pos and pos + history (so the last `history` changes are
// always one contiguous run); then m_prev_j = m_j.  sh: 8 floats of LDS.
template <int R, bool COH, class VS, class VC>
__device__ __forceinline__ void pred_modes(const PredStepArgs &a, int j0, int dj, int nr, bool push, int pos, VS s,
                                           VC c, float *sh) {
  // every row's own values, issued before the row loads by every thread (rows
  // past nr read row nr - 1), so that no load waits inside a branch
  float mp[R], mu[R], is[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = j0 + min(r, nr - 1) * dj;
    mp[r] = a.m_prev[j];
    mu[r] = a.mean[j];
    is[r] = a.inv_std[j];
  }
  float ps[R], pc[R];
  rows_part_f32<256, 8, R>(a.P + (int64_t)j0 * a.ldp, (int64_t)dj * a.ldp, nr, s, a.n_slopes, threadIdx.x, ps);
  rows_part_f32<256, 8, R>(a.PD + (int64_t)j0 * a.ldd, (int64_t)dj * a.ldd, nr, c, a.n_act, threadIdx.x, pc);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r >= nr) break;
    const float2 t = block_sum2(ps[r], pc[r], sh);
    if (threadIdx.x == 0) {
      const int j = j0 + r * dj;
      const float mj = t.x + t.y;
      if (push) {
        const float z = (mj - mp[r] - mu[r]) * is[r];
        put<COH>(a.hist + (int64_t)pos * a.n_modes + j, z);
        put<COH>(a.hist + (int64_t)(pos + a.history) * a.n_modes + j, z);
      }
      a.m_prev[j] = mj;
      a.m[j] = mj;
    }
  }
}

// Step 2 for hidden units i = i0 + r di, by a 256-thread workgroup: h_i =
// GELU(W1_i bf16(window) + b1_i), the window being the ring's slots pos + 1
// .. pos + history, oldest first.  sh: 4 R floats of LDS.
template <bool VEC, int R, bool COH, class VW>
__device__ __forceinline__ void pred_hidden(const PredStepArgs &a, int i0, int di, int nr, VW window, float *sh) {
  float z[R], b1[R];
#pragma unroll
  for (int r = 0; r < R; ++r) b1[r] = a.b1[i0 + min(r, nr - 1) * di];
  rows_dot_bf16<VEC, R>(a.W1 + (int64_t)i0 * a.n_in, (int64_t)di * a.n_in, nr, window, a.n_in, sh, z);
  if (threadIdx.x == 0)
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r < nr) put<COH>(a.h + i0 + r * di, gelu(z[r] + b1[r]));
}

// Step 3 for modes j = j0 + r dj, by a 256-thread workgroup: y_j = W2_j
// bf16(h) + b2_j, the forecast change d_j = y_j std_j + mean_j (0 before the
// window is full) and the forecast mode m_j + d_j.  sh: 4 R floats of LDS.
template <bool VEC, int R, bool COH, class VH>
__device__ __forceinline__ void pred_forecast(const PredStepArgs &a, int j0, int dj, int nr, bool full, VH h,
                                              float *sh) {
  float y[R], b2[R], sd[R], mn[R], mm[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {                 // issued before the row loads (rows past nr: row nr - 1)
    const int j = j0 + min(r, nr - 1) * dj;
    y[r] = 0.f;
    b2[r] = a.b2[j];
    sd[r] = a.std_[j];
    mn[r] = a.mean[j];
    mm[r] = a.m[j];
  }
  if (full) rows_dot_bf16<VEC, R>(a.W2 + (int64_t)j0 * a.n_hid, (int64_t)dj * a.n_hid, nr, h, a.n_hid, sh, y);
  if (threadIdx.x == 0)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r >= nr) break;
      const int j = j0 + r * dj;
      const float yj = full ? y[r] + b2[r] : 0.f;
      const float dv = full ? fmaf(yj, sd[r], mn[r]) : 0.0f;
      const float mj = mm[r];
      put<COH>(a.d + j, dv);
      if (a.modes_out != nullptr) {
        a.modes_out[j] = mj;
        a.modes_out[a.n_modes + j] = mj + dv;
      }
    }
}

// Step 4 for slopes i = i0 + r di, by one wavefront: out[r] = s_i + (P^T)_i d
// / gain (rows zero-padded to a multiple of 4; lane l takes the chunks l, l +
// 64, ...).
template <int R, class VD, class VS>
__device__ __forceinline__ void pred_slopes(const PredStepArgs &a, int i0, int di, int nr, int lane, VD d, VS s,
                                            float (&out)[R]) {
  float t[R], si[R];
#pragma unroll
  for (int r = 0; r < R; ++r) si[r] = s(i0 + min(r, nr - 1) * di);   // rows past nr: row nr - 1
  rows_part_f32<64, 2, R>(a.PT + (int64_t)i0 * a.ldt, (int64_t)di * a.ldt, nr, d, a.n_modes, lane, t);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float v = wave_total(t[r]) * a.inv_gain;
    out[r] = si[r] + v;
  }
}

}  // namespace rtcm
