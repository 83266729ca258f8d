// Device helpers shared by the kernel sources: the centre-of-gravity
// arithmetic of one subaperture and the fixed-order wavefront sum.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rtc_kernels.h"

namespace rtck {
namespace {

// Exact error-free transformations in float64 (round to nearest): a + b =
// s + e and a * b = p + e exactly.  The _rn intrinsics keep the compiler from
// contracting or reassociating them.
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
  s = __dadd_rn(a, b);
  const double bb = __dsub_rn(s, a);
  e = __dadd_rn(__dsub_rn(a, __dsub_rn(s, bb)), __dsub_rn(b, bb));
}
__device__ __forceinline__ void two_prod(double a, double b, double &p, double &e) {
  p = __dmul_rn(a, b);
  e = __fma_rn(a, b, -p);
}

// Adds x to the nonoverlapping expansion h[0..m) (increasing magnitude, zeros
// allowed) in place, the new largest component going to h[m] (Shewchuk's
// expansion growth): the sum of the components stays exact.
template <int M>
__device__ __forceinline__ void grow_expansion(double (&h)[5], double x) {
  double q = x;
#pragma unroll
  for (int i = 0; i < M; ++i) {
    double t;
    two_sum(q, h[i], q, t);
    h[i] = t;
  }
  h[M] = q;
}

// Exact decision for one pixel whose float64 estimate lay within rounding of
// the threshold (only possible when raw - dark is not exact in float64, i.e.
// the dark is outside {0} U [2^-13, 2^24) in magnitude): raw - dark = s + e and
// s flat, e flat are split exactly into two float64 terms each, so the excess
// (raw - dark) * flat - T is an exact sum of five float64 terms; the sum is
// grown into a nonoverlapping expansion, whose sign is that of its largest
// nonzero component.  r and x get float64 values of the excess and of
// (raw - dark) * flat; returns whether the excess is > 0.
__device__ __forceinline__ bool exact_excess(uint32_t raw, float dark, float flat, double T, double &r, double &x) {
  const double f = (double)flat;
  double s, e, p, pe, q, qe;
  two_sum((double)raw, -(double)dark, s, e);
  two_prod(s, f, p, pe);
  two_prod(e, f, q, qe);
  double h[5];
  h[0] = qe;
  grow_expansion<1>(h, q);
  grow_expansion<2>(h, pe);
  grow_expansion<3>(h, p);
  grow_expansion<4>(h, -T);
  int sign = 0;
#pragma unroll
  for (int i = 0; i < 5; ++i) sign = h[i] > 0.0 ? 1 : (h[i] < 0.0 ? -1 : sign);
  r = (((h[0] + h[1]) + h[2]) + h[3]) + h[4];
  x = ((qe + q) + pe) + p;
  return sign > 0;
}

// Value of a pixel in the weighted sums: mode 1 (subtract) the excess above the
// threshold, mode 2 (zero) the calibrated value above it, else 0; mode 0
// (none) the calibrated value of every pixel.
__device__ __forceinline__ double pixel_value(int mode, bool above, double r, double x) {
  return mode == 0 ? x : (above ? (mode == 1 ? r : x) : 0.0);
}

// Dark, flat and threshold of one pixel row (lane i of a tile with n pixels a
// side): its weighted sum S and x moment Sx, and the count of pixels above the
// threshold.  The decision uses r = fma(raw - dark, flat, -T) in float64,
// whose sign is exact when raw - dark is, i.e. when every dark of the
// calibration is 0 or of magnitude in [2^-13, 2^24) (FAST).  Otherwise
// (!FAST) a pixel whose r lies within the rounding bound of zero is marked,
// and after the row the marked pixels are fetched again
// (fetch(j, raw, dark, flat)) and decided by exact_excess, their
// contributions replacing the provisional ones; the row loop itself keeps only
// the mask.  The kernels that keep matrix rows in registers are built FAST
// only (their register budget has no room for the exact path).
// jz: 0, passed opaque by persistent kernels so that the column coordinates
// (double)j are formed in the loop instead of held in scalar registers.
template <int GS, bool FAST, class Fetch>
__device__ __forceinline__ void tile_row_sums(const uint32_t (&raw)[GS], const float2 (&cf)[GS], int n, float thr,
                                              int mode, double half, double &S, double &Sx, int &cnt,
                                              Fetch fetch, int jz = 0) {
  const double T = (double)thr;
  uint32_t amb = 0;
#pragma unroll
  for (int j = 0; j < GS; ++j) {
    if (j < n) {
      const double d = (double)raw[j] - (double)cf[j].x;
      const double f = (double)cf[j].y;
      const double r = fma(d, f, -T);
      const bool above = r > 0.0;
      if constexpr (!FAST) {
        // |exact - r| <= 2^-53 (|d f| + |r|) (1 + 2^-52) when raw - dark was rounded
        if (!(fabs(r) > 0x1p-50 * (fabs(d * f) + fabs(r)))) amb |= 1u << j;
      }
      const double v = pixel_value(mode, above, r, d * f);
      S += v;
      Sx = fma((double)(j + jz) - half, v, Sx);
      cnt += above ? 1 : 0;
    }
  }
  if constexpr (!FAST) {
    while (amb != 0u) {                            // rare: a dark outside the fast domain near a tie
      const int j = __builtin_ctz(amb);
      amb &= amb - 1u;
      uint32_t rj;
      float dk, fl;
      fetch(j, rj, dk, fl);
      const double d = (double)rj - (double)dk, f = (double)fl;
      const double r = fma(d, f, -T);
      const bool ap = r > 0.0;
      double re, xe;
      const bool ae = exact_excess(rj, dk, fl, T, re, xe);
      const double dv = pixel_value(mode, ae, re, xe) - pixel_value(mode, ap, r, d * f);
      S += dv;
      Sx = fma((double)j - half, dv, Sx);
      cnt += (ae ? 1 : 0) - (ap ? 1 : 0);
    }
  }
}

// The FAST form (no second fetch).
struct NoFetch {
  __device__ void operator()(int, uint32_t &, float &, float &) const {}
};
template <int GS>
__device__ __forceinline__ void tile_row_sums(const uint32_t (&raw)[GS], const float2 (&cf)[GS], int n, float thr,
                                              int mode, double half, double &S, double &Sx, int &cnt, int jz = 0) {
  tile_row_sums<GS, true>(raw, cf, n, thr, mode, half, S, Sx, cnt, NoFetch{}, jz);
}

// Tile sums over its GS lanes (butterfly: identical sums in every lane) and
// the centre of gravity relative to the tile centre (0 unless the weighted
// sum is positive).
template <int GS>
__device__ __forceinline__ void tile_centroid(double S, double Sx, int cnt, int i, double half, double &cx,
                                              double &cy, int &cnt_out) {
  double Sy = ((double)i - half) * S;
#pragma unroll
  for (int off = GS / 2; off > 0; off >>= 1) {
    S += __shfl_xor(S, off, GS);
    Sx += __shfl_xor(Sx, off, GS);
    Sy += __shfl_xor(Sy, off, GS);
    cnt += __shfl_xor(cnt, off, GS);
  }
  cx = 0.0;
  cy = 0.0;
  if (S > 0.0) {                     // thresholded modes: S > 0 exactly when a pixel is above
    cx = Sx / S;
    cy = Sy / S;
  }
  cnt_out = cnt;
}

// Wavefront sum without LDS traffic: DPP adds inside each row of 16 lanes
// (pairs, quads, half-row mirror, row mirror: every lane of a row ends with the
// row sum), then the four row sums read into scalars and added in a fixed
// order.  Needs all 64 lanes active; every lane returns the same total.
template <int CTRL>
__device__ __forceinline__ float dpp_read(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float row16_sum(float v) {
  v += dpp_read<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_read<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_read<0x141>(v);   // row_half_mirror
  v += dpp_read<0x140>(v);   // row_mirror
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
  v = row16_sum(v);
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
  return (r0 + r1) + (r2 + r3);
}

// Storage formats of the control matrix: a 16-byte chunk of codes decodes to
// EPC float32 values (exactly; the per-row scale is applied to the row sum).
template <int FMT>
struct Codec;
template <>
struct Codec<0> {                                 // float32
  static constexpr int EPC = 4;
  __device__ __forceinline__ static void decode(const uint4 &c, float (&v)[EPC]) {
    v[0] = __uint_as_float(c.x);
    v[1] = __uint_as_float(c.y);
    v[2] = __uint_as_float(c.z);
    v[3] = __uint_as_float(c.w);
  }
};
template <>
struct Codec<1> {                                 // IEEE binary16
  static constexpr int EPC = 8;
  __device__ __forceinline__ static void decode(const uint4 &c, float (&v)[EPC]) {
    const uint32_t w[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[2 * i] = (float)__builtin_bit_cast(_Float16, (uint16_t)(w[i] & 0xffffu));
      v[2 * i + 1] = (float)__builtin_bit_cast(_Float16, (uint16_t)(w[i] >> 16));
    }
  }
};
template <>
struct Codec<2> {                                 // bfloat16: the high half of a float32
  static constexpr int EPC = 8;
  __device__ __forceinline__ static void decode(const uint4 &c, float (&v)[EPC]) {
    const uint32_t w[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[2 * i] = __uint_as_float(w[i] << 16);
      v[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
    }
  }
};
template <>
struct Codec<3> {                                 // OCP FP8 E4M3 (e4m3fn)
  static constexpr int EPC = 16;
  __device__ __forceinline__ static void decode(const uint4 &c, float (&v)[EPC]) {
    typedef float f2v __attribute__((ext_vector_type(2)));
    const uint32_t w[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const f2v lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], false);   // bytes 0, 1
      const f2v hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], true);    // bytes 2, 3
      v[4 * i] = lo.x;
      v[4 * i + 1] = lo.y;
      v[4 * i + 2] = hi.x;
      v[4 * i + 3] = hi.y;
    }
  }
};

// ---------------------------------------------------------------------------
// Grid synchronisation of the persistent kernels: stage stamps, bounded waits,
// the per-frame barrier and the frame end stamp.
// ---------------------------------------------------------------------------
namespace sl = sync_layout;

// Stage stamp of the first trace_groups workgroups (thread 0) for the first
// trace_frames frames.
__device__ __forceinline__ void trace_stamp(const PersistArgs &p, int f, int stage) {
  if (p.trace != nullptr && f < p.trace_frames && (int)blockIdx.x < p.trace_groups && threadIdx.x == 0)
    p.trace[((int64_t)f * p.trace_groups + blockIdx.x) * kTraceStages + stage] = wall_clock64();
}

__device__ __forceinline__ bool bounded_wait(const PersistArgs &p, const uint32_t *word, uint32_t target) {
  int32_t spins = 0;
  while ((int32_t)(__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
    __builtin_amdgcn_s_sleep(1);
    if (++spins > p.spin_limit) {
      __hip_atomic_store(p.abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(p.sticky, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
  }
  return true;
}

// Wavefront 0 of every workgroup: waits until the external trigger releases
// frame f.  Lane 0 of workgroup 0 polls the host word (system scope) and the
// wavefront relays the value to every workgroup's mailbox line; the others
// poll their own line.  An expired wait raises the abort flag.
__device__ __forceinline__ void trigger_wait(const PersistArgs &p, int f) {
  const uint32_t target = p.trig_base + (uint32_t)f + 1u;
  if (blockIdx.x == 0) {
    int ok = 1;
    if (threadIdx.x == 0) {
      int32_t spins = 0;
      while ((int32_t)(__hip_atomic_load(p.trig_release, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) - target) <
             0) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > p.spin_limit) {
          __hip_atomic_store(p.abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(p.sticky, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
    }
    if (__builtin_amdgcn_readfirstlane(ok))
      for (uint32_t i = threadIdx.x + 1; i < gridDim.x; i += 64)
        __hip_atomic_store(p.bar + sl::kMailbox + 16 * i + 4, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else if (threadIdx.x == 0) {
    (void)bounded_wait(p, p.bar + sl::kMailbox + 16 * blockIdx.x + 4, target);
  }
}

// After this workgroup's commands of frame f are stored: the last workgroup to
// get here writes the frame's number to the trigger's done word.
__device__ __forceinline__ void trigger_done(const PersistArgs &p, int f) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t prev = __hip_atomic_fetch_add(p.bar + sl::kTrigDone, 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    if (prev == gridDim.x * (uint32_t)(f + 1) - 1u)
      __hip_atomic_store(p.trig_done, p.trig_base + (uint32_t)f + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// False when this workgroup's wait for the release expired (the abort flag is
// then raised): the frame's slopes may be incomplete, so the caller must not
// use them.  sh_flag: a shared word of the workgroup, left at bit 0 = this
// wait expired, bit 1 = stop after this frame (the abort flag was raised
// before this workgroup arrived, or by this wait).
// during(): loads that do not depend on the frame's slopes, issued by the
// wavefronts other than 0 while wavefront 0 arrives and waits (its arrival
// and polls wait for all of its own loads); the workgroup barrier at the end
// waits for them only if they write LDS.
template <class During>
__device__ __forceinline__ bool frame_barrier(const PersistArgs &p, uint32_t epoch, int f, uint32_t *sh_flag,
                                              During &&during) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wavefront's stores are complete
  __syncthreads();
  trace_stamp(p, f, 6);
  if (threadIdx.x >= 64) during();
  if (threadIdx.x < 64) {
    const uint32_t G = gridDim.x;
    int release = 0;
    uint32_t ab = 0;
    if (threadIdx.x == 0) {
      // the abort flag, read beside the arrival so that its round trip is the arrival's
      ab = __hip_atomic_load(p.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint32_t grp = blockIdx.x % sl::kGroups;
      const uint32_t per = (G - grp + sl::kGroups - 1) / sl::kGroups;   // workgroups in this group
      const uint32_t ngrp = G < (uint32_t)sl::kGroups ? G : (uint32_t)sl::kGroups;
      const uint32_t prev = __hip_atomic_fetch_add(p.bar + sl::kStride * grp, 1u, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
      trace_stamp(p, f, 7);
      if (prev == epoch * per - 1) {
        const uint32_t top = __hip_atomic_fetch_add(p.bar + sl::kTop, 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        release = top == epoch * ngrp - 1;
      }
    }
    if (__builtin_amdgcn_readfirstlane(release)) {
      for (uint32_t i = threadIdx.x; i < G; i += 64)
        __hip_atomic_store(p.bar + sl::kMailbox + 16 * i, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x == 0)
      *sh_flag = bounded_wait(p, p.bar + sl::kMailbox + 16 * blockIdx.x, epoch) ? (ab != 0u ? 2u : 0u) : 3u;
  }
  __syncthreads();
  return (*sh_flag & 1u) == 0u;
}

__device__ __forceinline__ bool frame_barrier(const PersistArgs &p, uint32_t epoch, int f, uint32_t *sh_flag) {
  return frame_barrier(p, epoch, f, sh_flag, [] {});
}

// End stamp of a frame: the latest of the per-workgroup end stamps (slot f
// mod `slots` of the end-stamp rows), reduced by the 64 lanes of one wavefront.
__device__ __forceinline__ void reduce_end_stamp(const PersistArgs &p, int f, int slots = 2) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t *ends = reinterpret_cast<const uint64_t *>(p.bar + sl::kEnds) + (f % slots) * sl::kMaxGroups;
  uint64_t m = 0;
  for (uint32_t i = lane; i < gridDim.x; i += 64) {
    const uint64_t v = __hip_atomic_load(ends + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    m = v > m ? v : m;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t o = __shfl_xor(m, d);
    m = o > m ? o : m;
  }
  if (lane == 0) p.ts[2 * (int64_t)f + 1] = m;
}


}  // namespace
}  // namespace rtck
