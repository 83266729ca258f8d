// gfx950 kernels of the SH-WFS real-time-control frame:
//   calib_cog_kernel       steps (a)-(b): dark, flat, threshold, centre of gravity
//   mvm_kernel             step  (c):     control matrix x slope vector (+ step (d) when unsplit)
//   reduce_integrate_kernel               fixed-order tree sum of split partials + step (d)
//
// Design notes (MI355X / CDNA4):
//  * The reconstruction streams the whole control matrix every frame and does
//    one FMA per 4 bytes: it is HBM/Infinity-Cache bound, not MFMA work, so it
//    is a VALU GEMV with 16-byte loads, the slope vector staged in LDS, and
//    float4 accumulators reduced by a 64-lane butterfly.
//  * Calibration + centroiding read ~4 MB per ELT frame.  One lane owns one
//    pixel row of one subaperture so a workgroup covers 256 / n_pix tiles;
//    per-row partial sums are combined in LDS in a fixed order.
//  * Everything is deterministic: no floating-point atomics, fixed reduction
//    trees, and the split-K partials are summed in a fixed pairwise tree.
#include "rtc_kernels.h"

namespace rtck {
namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// (a)-(b) calibration + centre of gravity
// ---------------------------------------------------------------------------
// MAXP >= n_pix: every row is loaded with fully unrolled, guarded loads so all
// of a lane's loads are in flight before the first use.
template <int MAXP>
__global__ __launch_bounds__(kBlock) void calib_cog_kernel(CalibArgs a) {
  __shared__ double sh_S[kBlock];
  __shared__ double sh_Sx[kBlock];
  __shared__ double sh_Sy[kBlock];
  __shared__ int sh_n[kBlock];

  const int tid = threadIdx.x;
  if (a.ts_start != nullptr && blockIdx.x == 0 && tid == 0) a.ts_start[0] = wall_clock64();

  const int n = a.n_pix;
  const int spb = kBlock / n;                    // subapertures per workgroup
  const int q = tid / n;                         // local subaperture
  const int i = tid - q * n;                     // pixel row inside the tile
  const int k = blockIdx.x * spb + q;
  const double half = 0.5 * (double)(n - 1);

  double S = 0.0, Sx = 0.0;
  int cnt = 0;
  if (q < spb && k < a.n_valid) {
    const uint16_t *prow = a.pix + (int64_t)a.tile_off[k] + (int64_t)i * a.W;
    const float2 *crow = a.calib + ((int64_t)k * n + i) * n;
    uint16_t raw[MAXP];
    float2 cf[MAXP];
#pragma unroll
    for (int j = 0; j < MAXP; ++j) {
      if (j < n) {
        raw[j] = prow[j];
        cf[j] = crow[j];
      }
    }
    const double T = (double)a.thr;
    const bool subtract = (a.mode == 1);
#pragma unroll
    for (int j = 0; j < MAXP; ++j) {
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
  sh_S[tid] = S;
  sh_Sx[tid] = Sx;
  sh_Sy[tid] = ((double)i - half) * S;
  sh_n[tid] = cnt;
  __syncthreads();

  if (tid < spb) {
    const int kk = blockIdx.x * spb + tid;
    if (kk < a.n_valid) {
      double tS = 0.0, tX = 0.0, tY = 0.0;
      int tn = 0;
      for (int r = 0; r < n; ++r) {            // rows in order: deterministic
        const int idx = tid * n + r;
        tS += sh_S[idx];
        tX += sh_Sx[idx];
        tY += sh_Sy[idx];
        tn += sh_n[idx];
      }
      double cx = 0.0, cy = 0.0;
      if (tn > 0) {
        cx = tX / tS;
        cy = tY / tS;
      }
      const float sx = (float)(cx - (double)a.ref[kk]);
      const float sy = (float)(cy - (double)a.ref[a.n_valid + kk]);
      a.s_int[kk] = sx;
      a.s_int[a.n_valid + kk] = sy;
      if (a.s_user != nullptr) {
        a.s_user[kk] = sx;
        a.s_user[a.n_valid + kk] = sy;
      }
      if (a.counts != nullptr) a.counts[kk] = tn;
    }
  }
}

// ---------------------------------------------------------------------------
// (c) reconstruction
// ---------------------------------------------------------------------------
__device__ __forceinline__ float wave_sum(float v) {
  // xor butterfly: every lane ends with the same (bitwise) total
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ float integrate_one(float *state, float *cmd, float *recon, int row,
                                               float a, float gain, float leak, float lo,
                                               float hi) {
  const float c0 = state[row];
  float c = fmaf(gain, a, leak * c0);
  c = fminf(fmaxf(c, lo), hi);
  state[row] = c;
  cmd[row] = c;
  if (recon != nullptr) recon[row] = a;
  return c;
}

// Completion stamp: the last workgroup to finish writes the end time once all
// workgroups' global writes are visible, then re-arms the counter.
__device__ __forceinline__ void completion_stamp(uint32_t *sync, uint64_t *ts_end) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t total = gridDim.x * gridDim.y;
    const uint32_t prev = atomicAdd(sync, 1u);
    if (prev == total - 1) {
      __threadfence();
      ts_end[0] = wall_clock64();
      atomicExch(sync, 0u);
    }
  }
}

// Workgroup = 4 wavefronts; wavefront w owns RPW consecutive actuator rows and
// streams them over this workgroup's slope partition (blockIdx.y).
template <int RPW>
__global__ __launch_bounds__(kBlock) void mvm_kernel(MvmArgs a, int32_t chunk4) {
  extern __shared__ float4 s_lds[];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int k0 = blockIdx.y * chunk4;
  const int nk = min(chunk4, a.n_s4 - k0);

  const float4 *s4 = reinterpret_cast<const float4 *>(a.s) + k0;
  for (int c = tid; c < nk; c += kBlock) s_lds[c] = s4[c];
  __syncthreads();

  const int row0 = (blockIdx.x * 4 + wave) * RPW;
  const float4 *rp[RPW];
  float4 acc[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    const int row = min(row0 + r, a.n_act - 1);   // clamp: loads stay in bounds
    rp[r] = reinterpret_cast<const float4 *>(a.R + (int64_t)row * a.ldr) + k0;
    acc[r] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
#pragma unroll 4
  for (int c = lane; c < nk; c += 64) {
    const float4 sv = s_lds[c];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const float4 rv = rp[r][c];
      acc[r].x = fmaf(rv.x, sv.x, acc[r].x);
      acc[r].y = fmaf(rv.y, sv.y, acc[r].y);
      acc[r].z = fmaf(rv.z, sv.z, acc[r].z);
      acc[r].w = fmaf(rv.w, sv.w, acc[r].w);
    }
  }
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    float v = (acc[r].x + acc[r].y) + (acc[r].z + acc[r].w);
    v = wave_sum(v);
    const int row = row0 + r;
    if (lane == 0 && row < a.n_act) {
      if (a.k_split > 1) {
        a.part[(int64_t)blockIdx.y * a.n_act + row] = v;
      } else {
        integrate_one(a.state, a.cmd, a.recon, row, v, a.gain, a.leak, a.cmd_min, a.cmd_max);
      }
    }
  }
  if (a.k_split == 1 && a.ts_end != nullptr) completion_stamp(a.sync, a.ts_end);
}

// Sum of the k_split partial actuator vectors in a fixed 64-leaf pairwise tree
// (missing leaves are 0), then the integrator.
__global__ __launch_bounds__(kBlock) void reduce_integrate_kernel(MvmArgs a) {
  const int row = blockIdx.x * kBlock + threadIdx.x;
  if (row < a.n_act) {
    float v[kMaxKSplit];
#pragma unroll
    for (int p = 0; p < kMaxKSplit; ++p)
      v[p] = (p < a.k_split) ? a.part[(int64_t)p * a.n_act + row] : 0.0f;
#pragma unroll
    for (int stride = 1; stride < kMaxKSplit; stride <<= 1) {
#pragma unroll
      for (int p = 0; p + stride < kMaxKSplit; p += 2 * stride) v[p] += v[p + stride];
    }
    integrate_one(a.state, a.cmd, a.recon, row, v[0], a.gain, a.leak, a.cmd_min, a.cmd_max);
  }
  if (a.ts_end != nullptr) completion_stamp(a.sync, a.ts_end);
}

// ---------------------------------------------------------------------------
// roofline probes
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void probe_copy_kernel(const float4 *__restrict__ src,
                                                            float4 *__restrict__ dst, int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(kBlock) void probe_read_kernel(const float4 *__restrict__ src,
                                                            int64_t n4, float *out) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  float acc = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += stride) {
    const float4 v = src[i];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  // keep the loads live; only a lane whose sum is exactly a sentinel writes
  if (acc == 1.2345e-30f) out[0] = acc;
}

}  // namespace

hipError_t launch_calib_cog(const CalibArgs &a, hipStream_t st) {
  if (a.n_pix < 1 || a.n_pix > 32) return hipErrorInvalidValue;
  const int spb = kBlock / a.n_pix;
  const int blocks = (a.n_valid + spb - 1) / spb;
  if (blocks == 0) return hipSuccess;
  if (a.n_pix <= 8)
    calib_cog_kernel<8><<<blocks, kBlock, 0, st>>>(a);
  else if (a.n_pix <= 16)
    calib_cog_kernel<16><<<blocks, kBlock, 0, st>>>(a);
  else
    calib_cog_kernel<32><<<blocks, kBlock, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_mvm_integrate(const MvmArgs &in, int32_t *used, hipStream_t st) {
  MvmArgs a = in;
  constexpr int RPW = 2;
  int ks = a.k_split < 1 ? 1 : (a.k_split > kMaxKSplit ? kMaxKSplit : a.k_split);
  const int min_ks = (a.n_s4 + kMaxChunk4 - 1) / kMaxChunk4;
  if (ks < min_ks) ks = min_ks;
  if (ks > kMaxKSplit) return hipErrorInvalidValue;
  int chunk4 = (a.n_s4 + ks - 1) / ks;
  if (chunk4 < 1) chunk4 = 1;
  ks = (a.n_s4 + chunk4 - 1) / chunk4;           // partitions actually populated
  if (ks < 1) ks = 1;
  if (ks > 1 && a.part == nullptr) return hipErrorInvalidValue;
  a.k_split = ks;
  if (used) *used = ks;
  const dim3 grid((a.n_act + 4 * RPW - 1) / (4 * RPW), ks);
  const size_t lds = (size_t)chunk4 * sizeof(float4);
  mvm_kernel<RPW><<<grid, kBlock, lds, st>>>(a, chunk4);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || ks == 1) return e;
  reduce_integrate_kernel<<<(a.n_act + kBlock - 1) / kBlock, kBlock, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_probe_copy(const void *src, void *dst, int64_t n_bytes, hipStream_t st) {
  const int64_t n4 = n_bytes / 16;
  if (n4 == 0) return hipSuccess;
  int64_t blocks = (n4 + kBlock * 4 - 1) / (kBlock * 4);
  if (blocks > 65536) blocks = 65536;
  probe_copy_kernel<<<(unsigned)blocks, kBlock, 0, st>>>(static_cast<const float4 *>(src),
                                                         static_cast<float4 *>(dst), n4);
  return hipGetLastError();
}

hipError_t launch_probe_read(const void *src, int64_t n_bytes, float *out, hipStream_t st) {
  const int64_t n4 = n_bytes / 16;
  if (n4 == 0) return hipSuccess;
  int64_t blocks = (n4 + kBlock * 4 - 1) / (kBlock * 4);
  if (blocks > 65536) blocks = 65536;
  probe_read_kernel<<<(unsigned)blocks, kBlock, 0, st>>>(static_cast<const float4 *>(src), n4, out);
  return hipGetLastError();
}

}  // namespace rtck
