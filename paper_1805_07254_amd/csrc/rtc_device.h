// Device helpers shared by the kernel sources: the centre-of-gravity
// arithmetic of one subaperture and the fixed-order wavefront sum.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rtc_kernels.h"

namespace rtck {
namespace {

// Dark, flat and threshold of one pixel row (lane i of a tile with n pixels a
// side): its weighted sum S and x moment Sx, and the count of pixels above
// the threshold.
template <int GS>
__device__ __forceinline__ void tile_row_sums(const uint32_t (&raw)[GS], const float2 (&cf)[GS], int n, float thr,
                                              bool subtract, double half, double &S, double &Sx, int &cnt) {
  const double T = (double)thr;
#pragma unroll
  for (int j = 0; j < GS; ++j) {
    if (j < n) {
      // raw - dark is exact in float64 for the accepted dark domain; the single
      // rounding of the fma keeps the sign of (raw - dark) * flat - T exact.
      const double d = (double)raw[j] - (double)cf[j].x;
      const double f = (double)cf[j].y;
      const double r = fma(d, f, -T);
      const bool above = r > 0.0;
      const double v = above ? (subtract ? r : d * f) : 0.0;
      S += v;
      Sx = fma((double)j - half, v, Sx);
      cnt += above ? 1 : 0;
    }
  }
}

// Tile sums over its GS lanes (butterfly: identical sums in every lane) and
// the centre of gravity relative to the tile centre (0 without a pixel above
// the threshold).
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
  if (cnt > 0) {
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

}  // namespace
}  // namespace rtck
