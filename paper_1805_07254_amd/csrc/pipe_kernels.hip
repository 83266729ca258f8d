// gfx950 kernels of pixel-stream processing: the in-launch camera emulator,
// the workers that process subapertures as their rows land, and the
// column-major copy of the control matrix they read.
#include "rtc_kernels.h"
#include "rtc_device.h"

namespace rtck {
namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// Pixel-stream frames (processing while the pixels arrive, Section 2.3.6 and
// Figure 6; latency as measured in Section 3.2).  The last workgroup emulates
// the camera:
// at each packet's scheduled time it copies the packet's rows from the source
// frame into the frame's ring slot with device-coherent word stores, waits
// for them to complete and publishes the landed-row count (rows of frame f
// count from f H on) in kRowCopies copies.  Every other workgroup is a worker
// (a thread of the paper's horizontal strategy): its subapertures are a
// contiguous run in arrival order, processed in passes of subapertures that
// need the same rows, each pass starting as soon as those rows have landed;
// pixels are read with device-coherent word loads, so neither side needs a
// cache write-back or invalidation.  A pass calibrates and centroids its
// subapertures and multiplies their slopes into the worker's packed matrix
// columns (column-major, thread t handles quads of 4 consecutive rows); the
// worker's trailing lds_cols columns -- the ones whose slopes arrive last --
// are copied to LDS once per launch.  The partial actuator vector is then
// published.  The actuator rows belong to the first n_own workers (owners),
// whose own subapertures land early: an owner adds the P partial vectors of
// its rows in worker order, each as soon as it is published, so only the last
// workers' vectors remain after the last pixel.  The tail subapertures (the
// last rows of the frame) are not allocated to workers: every owner
// calibrates them itself and applies their columns (kept in LDS) to its own
// rows, so after the last pixel nothing travels between workgroups.  Every
// wait is bounded in time and gives up when another workgroup has raised the
// abort flag, so every workgroup exits.
// ---------------------------------------------------------------------------
namespace pl = pipe_layout;
constexpr int kPipeQ = pl::kMaxQuadsPerThread;

// Four consecutive codes of a packed column, decoded to float32.
template <int FMT>
struct Quad;
template <>
struct Quad<0> {
  using T = float4;
  __device__ __forceinline__ static float4 get(const T &c) { return c; }
};
template <>
struct Quad<1> {
  using T = uint2;
  __device__ __forceinline__ static float4 get(const T &c) {
    return make_float4((float)__builtin_bit_cast(_Float16, (uint16_t)(c.x & 0xffffu)),
                       (float)__builtin_bit_cast(_Float16, (uint16_t)(c.x >> 16)),
                       (float)__builtin_bit_cast(_Float16, (uint16_t)(c.y & 0xffffu)),
                       (float)__builtin_bit_cast(_Float16, (uint16_t)(c.y >> 16)));
  }
};
template <>
struct Quad<2> {
  using T = uint2;
  __device__ __forceinline__ static float4 get(const T &c) {
    return make_float4(__uint_as_float(c.x << 16), __uint_as_float(c.x & 0xffff0000u), __uint_as_float(c.y << 16),
                       __uint_as_float(c.y & 0xffff0000u));
  }
};
template <>
struct Quad<3> {
  using T = uint32_t;
  __device__ __forceinline__ static float4 get(const T &c) {
    typedef float f2v __attribute__((ext_vector_type(2)));
    const f2v lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)c, false);
    const f2v hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)c, true);
    return make_float4(lo.x, lo.y, hi.x, hi.y);
  }
};

__device__ __forceinline__ void pipe_raise_abort(const PipeArgs &p) {
  __hip_atomic_store(p.abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(p.sticky, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One thread waits until *word - target >= 0 (wrapping).  False when the wait
// exceeded p.wait_ticks (the abort flags are then raised) or another
// workgroup raised the abort flag.
__device__ bool pipe_wait(const PipeArgs &p, const uint32_t *word, uint32_t target) {
  const uint64_t t0 = wall_clock64();
  for (uint32_t spins = 0;; ++spins) {
    if ((int32_t)(__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) >= 0) return true;
    __builtin_amdgcn_s_sleep(2);
    if ((spins & 31) == 31) {
      if (__hip_atomic_load(p.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
      if (wall_clock64() - t0 > (uint64_t)p.wait_ticks) {
        pipe_raise_abort(p);
        return false;
      }
    }
  }
}

// The whole workgroup waits (thread 0 polls); uniform result.
__device__ bool pipe_block_wait(const PipeArgs &p, const uint32_t *word, uint32_t target, uint32_t *sh) {
  if (threadIdx.x == 0) *sh = pipe_wait(p, word, target) ? 1u : 0u;
  __syncthreads();
  const bool ok = *sh != 0;
  __syncthreads();
  return ok;
}

// Camera workgroup.
__device__ void pipe_camera(const PipeArgs &p, int P, uint32_t *sh_flag, uint64_t *sh_t0) {
  const int tid = threadIdx.x;
  if (tid == 0) *sh_t0 = wall_clock64() + (uint64_t)p.lead;
  __syncthreads();
  const uint64_t T0 = *sh_t0;
  const uint32_t *src_w = reinterpret_cast<const uint32_t *>(p.src);
  uint32_t *ring_w = reinterpret_cast<uint32_t *>(p.ring);
  const int64_t n_words = p.frame_elems / 2;
  for (int f = 0; f < p.n_frames; ++f) {
    // slot f & 1 held frame f - 2: every worker must be done with it
    if (f >= 2 && !pipe_block_wait(p, p.sync + pl::kOwnDone, (uint32_t)(P * (f - 1)), sh_flag)) return;
    const double fbase = (double)f * p.t_frame;
    const uint32_t *sw = src_w + (int64_t)f * (p.src_stride / 2);
    uint32_t *dw = ring_w + (int64_t)(f & 1) * (p.ring_stride / 2);
    uint64_t first = 0, last = 0, slip = 0;
    for (int i0 = 0; i0 < p.H; i0 += p.rows_per_packet) {
      const int i1 = min(i0 + p.rows_per_packet, p.H);
      const uint64_t sched = T0 + (uint64_t)(fbase + (double)i1 * p.t_row);
      if (tid == 0) {
        uint32_t stop = 0;
        for (uint32_t spins = 0; wall_clock64() < sched; ++spins) {
          __builtin_amdgcn_s_sleep(2);
          if ((spins & 31) == 31 && __hip_atomic_load(p.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            stop = 1;
            break;
          }
        }
        *sh_flag = stop;
      }
      __syncthreads();
      const bool stop = *sh_flag != 0;
      __syncthreads();
      if (stop) return;
      const int64_t w0 = ((int64_t)i0 * p.W) / 2;
      const int64_t w1 = min(n_words, ((int64_t)i1 * p.W + 1) / 2);
      for (int64_t w = w0 + tid; w < w1; w += 512)
        __hip_atomic_store(dw + w, sw[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wavefront's rows are in memory
      __syncthreads();
      if (tid == 0) {
        const uint64_t now = wall_clock64();
        slip = (now - sched) > slip ? (now - sched) : slip;
        if (i0 == 0) first = now;
        last = now;
      }
      if (tid < pl::kRowCopies)
        __hip_atomic_store(p.sync + tid * pl::kStride, (uint32_t)((int64_t)f * p.H + i1), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tid == 0 && p.cam_ts != nullptr) {
      uint64_t *ts = p.cam_ts + (int64_t)f * pl::kCamStamps;
      ts[0] = T0 + (uint64_t)fbase;
      ts[1] = first;
      ts[2] = last;
      ts[3] = slip;
    }
  }
}

// What a calibration pass needs besides the pixels, loaded before the wait for
// its rows: lane i of tile jj = j + tid / GS holds the tile, its row's (dark,
// flat) pairs and, in lane 0, the reference slopes.
template <int GS>
struct PassPrefetch {
  TileDesc t;
  float2 cf[GS];
  float rx, ry;
  bool valid;
};

template <int GS>
__device__ __forceinline__ void pipe_pass_prefetch(const PipeArgs &p, int k0, int j, int j2, PassPrefetch<GS> &pf) {
  const int tid = threadIdx.x;
  const int jj = j + tid / GS;
  const int i = tid & (GS - 1);
  pf.valid = jj < j2;
  pf.t = TileDesc{};
  pf.rx = pf.ry = 0.f;
  if (pf.valid) pf.t = p.tiles[k0 + jj];
  const int n = pf.t.n;
  if (pf.valid && i < n) {
    const float2 *crow = p.calib + (int64_t)pf.t.calib_off + (int64_t)i * n;
#pragma unroll
    for (int x = 0; x < GS; ++x)
      if (x < n) pf.cf[x] = crow[x];
  }
  if (pf.valid && i == 0) {
    pf.rx = p.ref[pf.t.sx];
    pf.ry = p.ref[pf.t.sy];
  }
}

// Calibration + centre of gravity of the pass's subapertures once their rows
// have landed: slopes of local subaperture jj to sh_s[2 jj], sh_s[2 jj + 1];
// with `outputs`, also to the caller's slope and count arrays.
template <int GS>
__device__ __forceinline__ void pipe_pass_finish(const PipeArgs &p, int f, const uint32_t *slot, int k0, int j,
                                                 const PassPrefetch<GS> &pf, float *sh_s, bool outputs) {
  const int tid = threadIdx.x;
  const int jj = j + tid / GS;
  const int i = tid & (GS - 1);
  const TileDesc &t = pf.t;
  const int n = t.n;
  const double half = 0.5 * (double)(n - 1);
  double S = 0.0, Sx = 0.0;
  int cnt = 0;
  if (pf.valid && i < n) {
    const int64_t e0 = (int64_t)t.off + (int64_t)i * t.pitch;
    const uint32_t *wp = slot + (e0 >> 1);
    const bool odd = (e0 & 1) != 0;
    constexpr int NW = GS / 2 + 1;
    const int nw = ((odd ? 1 : 0) + n + 1) >> 1;     // words covering the row's n pixels
    uint32_t w[NW];
#pragma unroll
    for (int q = 0; q < NW; ++q)
      w[q] = q < nw ? __hip_atomic_load(wp + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
    uint32_t raw[GS];
#pragma unroll
    for (int q = 0; q < GS / 2; ++q) {
      raw[2 * q] = odd ? (w[q] >> 16) : (w[q] & 0xffffu);
      raw[2 * q + 1] = odd ? (w[q + 1] & 0xffffu) : (w[q] >> 16);
    }
    tile_row_sums<GS>(raw, pf.cf, n, t.thr, p.mode, half, S, Sx, cnt);
  }
  double cx, cy;
  tile_centroid<GS>(S, Sx, cnt, i, half, cx, cy, cnt);
  if (pf.valid && i == 0) {
    const float sx = (float)(cx - (double)pf.rx);
    const float sy = (float)(cy - (double)pf.ry);
    sh_s[2 * jj] = sx;
    sh_s[2 * jj + 1] = sy;
    if (outputs) {
      if (p.s_user != nullptr) {
        float *su = p.s_user + (int64_t)f * 2 * p.n_valid;
        su[t.sx] = sx;
        su[t.sy] = sy;
      }
      if (p.counts != nullptr) p.counts[(int64_t)f * p.n_valid + k0 + jj] = cnt;
    }
  }
}

// acc += columns [c0, c1) of cols (column c at cols + (c - cbase) nq) times
// sh_s[c], in column order; U columns' loads in flight.
template <int FMT>
__device__ __forceinline__ void pipe_columns(const typename Quad<FMT>::T *cols, int64_t nq, int c0, int c1, int cbase,
                                             const float *sh_s, float4 (&acc)[kPipeQ]) {
  using QT = typename Quad<FMT>::T;
  constexpr int U = FMT == 0 ? 4 : 8;
  const int tid = threadIdx.x;
  for (int c = c0; c < c1; c += U) {
    QT m[U][kPipeQ];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int i = 0; i < kPipeQ; ++i) {
        const int64_t q = tid + 512 * i;
        m[u][i] = (c + u < c1 && q < nq) ? cols[(int64_t)(c + u - cbase) * nq + q] : QT{};
      }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (c + u < c1) {
        const float s = sh_s[c + u];
#pragma unroll
        for (int i = 0; i < kPipeQ; ++i) {
          const float4 v = Quad<FMT>::get(m[u][i]);
          acc[i].x = fmaf(v.x, s, acc[i].x);
          acc[i].y = fmaf(v.y, s, acc[i].y);
          acc[i].z = fmaf(v.z, s, acc[i].z);
          acc[i].w = fmaf(v.w, s, acc[i].w);
        }
      }
    }
  }
}

// One code of a packed column, decoded.
template <int FMT>
__device__ __forceinline__ float decode_one(const void *packed, int64_t idx) {
  if constexpr (FMT == 0) {
    return static_cast<const float *>(packed)[idx];
  } else if constexpr (FMT == 1) {
    return (float)__builtin_bit_cast(_Float16, static_cast<const uint16_t *>(packed)[idx]);
  } else if constexpr (FMT == 2) {
    return __uint_as_float((uint32_t)static_cast<const uint16_t *>(packed)[idx] << 16);
  } else {
    typedef float f2v __attribute__((ext_vector_type(2)));
    const f2v v = __builtin_amdgcn_cvt_pk_f32_fp8((int)static_cast<const uint8_t *>(packed)[idx], false);
    return v.x;
  }
}

// Calibration passes over local subapertures [j0, j1) of the run starting at
// k0 (need[] local to the run), each pass starting when its rows have landed;
// after each pass, `after(j, j2)` runs with the pass's slopes in sh_s.
// False when a wait gave up.
template <int GS, typename After>
__device__ __forceinline__ bool pipe_passes(const PipeArgs &p, int f, const uint32_t *slot, const uint32_t *rows_ctr,
                                            int k0, int j0, int j1, const int32_t *need, float *sh_s, bool outputs,
                                            uint32_t *sh_wait, After after) {
  constexpr int SPP = 512 / GS;
  for (int j = j0; j < j1;) {
    const int nd = need[j];
    int j2 = j + 1;
    while (j2 < j1 && j2 < j + SPP && need[j2] == nd) ++j2;
    PassPrefetch<GS> pf;
    pipe_pass_prefetch<GS>(p, k0, j, j2, pf);
    if (!pipe_block_wait(p, rows_ctr, (uint32_t)((int64_t)f * p.H + nd), sh_wait)) return false;
    pipe_pass_finish<GS>(p, f, slot, k0, j, pf, sh_s, outputs);
    __syncthreads();
    after(j, j2);
    j = j2;
  }
  return true;
}

template <int FMT, int GS>
__global__ __launch_bounds__(512) void pipe_kernel(PipeArgs p) {
  using QT = typename Quad<FMT>::T;
  // LDS: [lds_cols][nq] codes, sh_s [2 max_nb], sh_need [max_nb], tail need [n_tail],
  // tail slopes [2 n_tail], tail matrix block [2 n_tail][own_max] floats
  extern __shared__ uint4 pipe_lds[];
  __shared__ uint32_t sh_abort, sh_wait;
  __shared__ uint64_t sh_t0;
  __shared__ float sh_red[8 * 64];                 // per-wavefront partial-vector sums of the owned rows
  __shared__ uint32_t sh_ok[8];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int P = (int)gridDim.x - 1;
  const int b = blockIdx.x;
  if (b == P) {
    pipe_camera(p, P, &sh_wait, &sh_t0);
    return;
  }
  const int64_t nq = p.ldp / 4;
  const int nt2 = 2 * p.n_tail;
  QT *lds_cols = reinterpret_cast<QT *>(pipe_lds);
  float *sh_s = reinterpret_cast<float *>(reinterpret_cast<char *>(pipe_lds) +
                                          (int64_t)p.lds_cols * nq * (int64_t)sizeof(QT));
  int32_t *sh_need = reinterpret_cast<int32_t *>(sh_s + 2 * p.max_nb);
  int32_t *sh_tneed = sh_need + p.max_nb;
  float *sh_ts = reinterpret_cast<float *>(sh_tneed + p.n_tail);
  float *sh_tR = sh_ts + nt2;
  const int k0 = p.first[b], nb = p.first[b + 1] - k0, ncol = 2 * nb;
  const int kt = p.n_valid - p.n_tail;             // first tail subaperture
  const int Lc = min(ncol, p.lds_cols), lfirst = ncol - Lc;
  const QT *gcols = reinterpret_cast<const QT *>(p.packed) + (int64_t)2 * k0 * nq;
  // owners are the first n_own workers (their own subapertures land first); owner b
  // holds actuator rows [ob, ob + nown), row ob + r in lane r of wavefront 0
  const bool owner = b < p.n_own;
  const int ob = owner ? (int)(((int64_t)b * p.n_act) / p.n_own) : 0;
  const int nown = owner ? (int)(((int64_t)(b + 1) * p.n_act) / p.n_own) - ob : 0;
  for (int64_t x = tid; x < (int64_t)Lc * nq; x += 512) lds_cols[x] = gcols[(int64_t)lfirst * nq + x];
  for (int j = tid; j < nb; j += 512) sh_need[j] = p.need[k0 + j];
  for (int j = tid; j < p.n_tail; j += 512) sh_tneed[j] = p.need[kt + j];
  for (int x = tid; x < nt2 * p.own_max; x += 512) {
    const int c = x / p.own_max, r = x - c * p.own_max;
    sh_tR[x] = r < nown ? decode_one<FMT>(p.packed, (int64_t)(2 * kt + c) * p.ldp + ob + r) : 0.f;
  }
  float st = (wave == 0 && lane < nown) ? p.state[ob + lane] : 0.f;
  __syncthreads();
  const uint32_t *rows_ctr = p.sync + (b % pl::kRowCopies) * pl::kStride;
  const uint32_t *ring_w = reinterpret_cast<const uint32_t *>(p.ring);
  const uint32_t *flags = p.sync + pl::kFlags;

  for (int f = 0; f < p.n_frames; ++f) {
    if (tid == 0) sh_abort = __hip_atomic_load(p.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const bool aborted = sh_abort != 0;
    __syncthreads();
    if (aborted) break;
    // partial slot f & 1 held frame f - 2, consumed by every owner before it counted
    // frame f - 2 done; by now that has long happened, so this wait returns at once
    if (f >= 2 && !pipe_block_wait(p, p.sync + pl::kOwnDone, (uint32_t)(P * (f - 1)), &sh_wait)) break;
    const uint32_t *slot = ring_w + (int64_t)(f & 1) * (p.ring_stride / 2);
    float4 acc[kPipeQ];
#pragma unroll
    for (int i = 0; i < kPipeQ; ++i) acc[i] = make_float4(0.f, 0.f, 0.f, 0.f);

    // (a)-(c) own subapertures, pass by pass as their rows land
    const bool ok_main = pipe_passes<GS>(p, f, slot, rows_ctr, k0, 0, nb, sh_need, sh_s, true, &sh_wait,
                                         [&](int j, int j2) {
      const int c0 = 2 * j, c1 = 2 * j2;
      if (c0 < lfirst) pipe_columns<FMT>(gcols, nq, c0, min(c1, lfirst), 0, sh_s, acc);
      if (c1 > lfirst) pipe_columns<FMT>(lds_cols, nq, max(c0, lfirst), c1, lfirst, sh_s, acc);
    });
    if (!ok_main) break;

    // publish the partial vector
    float *part_f = p.part + (int64_t)(f & 1) * P * p.ldp;
    {
      uint64_t *dst = reinterpret_cast<uint64_t *>(part_f + (int64_t)b * p.ldp);
#pragma unroll
      for (int i = 0; i < kPipeQ; ++i) {
        const int64_t q = tid + 512 * i;
        if (q < nq) {
          const uint64_t lo = (uint64_t)__float_as_uint(acc[i].x) | ((uint64_t)__float_as_uint(acc[i].y) << 32);
          const uint64_t hi = (uint64_t)__float_as_uint(acc[i].z) | ((uint64_t)__float_as_uint(acc[i].w) << 32);
          __hip_atomic_store(dst + 2 * q, lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(dst + 2 * q + 1, hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (tid == 0) {
      if (p.wk_ts != nullptr) p.wk_ts[((int64_t)f * P + b) * 2] = wall_clock64();
      __hip_atomic_store(p.sync + pl::kFlags + 16 * b, (uint32_t)(f + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }

    if (owner) {
      // (c) own rows: the P partial vectors, each added as soon as it is published.
      // Wavefront k adds workers k, k + 8, k + 16, ... in order (lanes = rows); the 8
      // sums are then added in wavefront order, so the order never depends on timing.
      float tot = 0.f, tail = 0.f;
      {
        float part_sum = 0.f;
        bool ok = true;
        const float *prow = part_f + ob + lane;
        uint64_t t_progress = wall_clock64();
        for (int w = wave, spins = 0; w < P;) {
          const int wl = w + 8 * lane;
          const bool ready = wl < P && (int32_t)(__hip_atomic_load(flags + 16 * wl, __ATOMIC_RELAXED,
                                                                   __HIP_MEMORY_SCOPE_AGENT) - (uint32_t)(f + 1)) >= 0;
          const uint64_t waiting = ~__ballot(ready);
          const int m = waiting == 0 ? 64 : (int)__builtin_ctzll(waiting);   // published run from w on
          if (m == 0) {
            __builtin_amdgcn_s_sleep(1);
            if ((++spins & 31) == 0) {
              int stop = 0;
              if (lane == 0) {
                if (__hip_atomic_load(p.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                  stop = 1;
                } else if (wall_clock64() - t_progress > (uint64_t)p.wait_ticks) {
                  pipe_raise_abort(p);
                  stop = 1;
                }
              }
              if (__builtin_amdgcn_readfirstlane(stop)) {
                ok = false;
                break;
              }
            }
            continue;
          }
          for (int i = 0; i < m; i += 16) {
            float v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u)
              v[u] = (i + u < m && lane < nown)
                         ? __hip_atomic_load(prow + (int64_t)(w + 8 * (i + u)) * p.ldp, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT)
                         : 0.f;
#pragma unroll
            for (int u = 0; u < 16; ++u)
              if (i + u < m) part_sum += v[u];
          }
          w += 8 * m;
          spins = 0;
          t_progress = wall_clock64();
        }
        sh_red[wave * 64 + lane] = part_sum;
        if (lane == 0) sh_ok[wave] = ok ? 1u : 0u;
      }
      __syncthreads();
      bool ok_sum = true;
#pragma unroll
      for (int k = 0; k < 8; ++k) ok_sum = ok_sum && sh_ok[k] != 0;
      if (wave == 0)
#pragma unroll
        for (int k = 0; k < 8; ++k) tot += sh_red[k * 64 + lane];
      __syncthreads();
      if (!ok_sum) break;

      // (a)-(c) tail subapertures: every owner calibrates them and applies their columns
      // to its own rows, pass by pass
      if (p.n_tail > 0) {
        const bool ok_tail = pipe_passes<GS>(p, f, slot, rows_ctr, kt, 0, p.n_tail, sh_tneed, sh_ts, b == 0,
                                             &sh_wait, [&](int j, int j2) {
          if (wave == 0 && lane < nown)
            for (int c = 2 * j; c < 2 * j2; ++c) tail = fmaf(sh_tR[c * p.own_max + lane], sh_ts[c], tail);
        });
        if (!ok_tail) break;
      }

      // (d) integrator of the owned rows
      if (wave == 0 && lane < nown) {
        const int row = ob + lane;
        float a = tot + tail;
        if (p.scales != nullptr) a *= p.scales[row];
        float c = fmaf(p.gain, a, p.leak * st);
        c = fminf(fmaxf(c, p.cmd_min), p.cmd_max);
        st = c;
        p.cmd[(int64_t)f * p.n_act + row] = c;
        if (p.recon != nullptr) p.recon[(int64_t)f * p.n_act + row] = a;
      }
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
    }
    if (tid == 0) {
      if (p.wk_ts != nullptr) p.wk_ts[((int64_t)f * P + b) * 2 + 1] = wall_clock64();
      __hip_atomic_fetch_add(p.sync + pl::kOwnDone, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (wave == 0 && lane < nown) p.state[ob + lane] = st;
}

// Zeroes the landed-row counters, the flags of P workers, the done counter and
// the abort flag (stores, not a memset).
__global__ __launch_bounds__(kBlock) void pipe_reset_kernel(uint32_t *sync, uint32_t *abort_flag, int P) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  uint32_t *w = nullptr;
  if (t < pl::kRowCopies) w = sync + pl::kStride * t;
  else if (t == pl::kRowCopies) w = sync + pl::kOwnDone;
  else if (t == pl::kRowCopies + 1) w = abort_flag;
  else if (t >= 64 && t < 64 + P) w = sync + pl::kFlags + 16 * (t - 64);
  if (w != nullptr) __hip_atomic_store(w, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Column-major copy of the matrix codes for the pixel-stream workers (64 x 64
// tiles transposed through LDS).
template <typename U>
__global__ __launch_bounds__(256) void pack_columns_kernel(const U *Rq, int64_t ldq, const TileDesc *tiles,
                                                           int n_valid, int n_act, U *packed, int64_t ldp) {
  __shared__ U tile[64][65];
  const int pc0 = blockIdx.x * 64;
  const int64_t r0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int pc = pc0 + tx;
  int sc = -1;
  if (pc < 2 * n_valid) {
    const TileDesc t = tiles[pc >> 1];
    sc = (pc & 1) ? t.sy : t.sx;
  }
  for (int rr = ty; rr < 64; rr += 4) {
    const int64_t r = r0 + rr;
    tile[rr][tx] = (sc >= 0 && r < n_act) ? Rq[r * ldq + sc] : U(0);
  }
  __syncthreads();
  for (int cc = ty; cc < 64; cc += 4) {
    const int pcw = pc0 + cc;
    const int64_t r = r0 + tx;
    if (pcw < 2 * n_valid && r < ldp) packed[(int64_t)pcw * ldp + r] = tile[tx][cc];
  }
}

}  // namespace

int format_code_bytes(int fmt) { return fmt == 0 ? 4 : (fmt == 3 ? 1 : 2); }

size_t pipe_lds_fixed(int max_nb, int n_tail, int own_max) {
  return sizeof(float) * ((size_t)3 * max_nb + (size_t)3 * n_tail + (size_t)2 * n_tail * own_max) + 16;
}

template <int FMT, int GS>
static hipError_t launch_pipe_variant(const PipeArgs &p, int G, size_t lds, hipStream_t st) {
  auto kern = pipe_kernel<FMT, GS>;
  int dev = 0, ncu = 0;
  hipError_t e;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds)) != hipSuccess)
    return e;
  int per_cu = 0;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 512, lds)) != hipSuccess) return e;
  if (per_cu * ncu < G) return hipErrorCooperativeLaunchTooLarge;
  const int P = G - 1;
  pipe_reset_kernel<<<(64 + P + kBlock - 1) / kBlock, kBlock, 0, st>>>(p.sync, p.abort_flag, P);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  PipeArgs pa = p;
  void *args[] = {&pa};
  e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kern), dim3(G), dim3(512), args, lds, st);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

template <int FMT>
static hipError_t launch_pipe_fmt(const PipeArgs &p, int G, size_t lds, hipStream_t st) {
  if (p.max_n <= 8) return launch_pipe_variant<FMT, 8>(p, G, lds, st);
  if (p.max_n <= 16) return launch_pipe_variant<FMT, 16>(p, G, lds, st);
  return launch_pipe_variant<FMT, 32>(p, G, lds, st);
}

hipError_t launch_pipe(const PipeArgs &p, int G, size_t lds, hipStream_t st) {
  if (p.n_frames <= 0) return hipSuccess;
  if (p.max_n < 1 || p.max_n > 32 || G < 2 || G - 1 > pl::kMaxWorkers) return hipErrorInvalidValue;
  if (p.ldp % 64 != 0 || p.ldp / 4 > (int64_t)kPipeQ * 512) return hipErrorInvalidValue;
  if (p.n_own < 1 || p.n_own > G - 1 || p.own_max > 64 || p.own_max < (p.n_act + p.n_own - 1) / p.n_own)
    return hipErrorInvalidValue;
  if (p.n_tail < 0 || p.n_tail > kPipeMaxTail || p.n_tail > p.n_valid) return hipErrorInvalidValue;
  if (p.frame_elems % 2 != 0 || p.src_stride % 2 != 0 || p.ring_stride % 128 != 0 || p.rows_per_packet < 1)
    return hipErrorInvalidValue;
  switch (p.fmt) {
    case 0: return launch_pipe_fmt<0>(p, G, lds, st);
    case 1: return launch_pipe_fmt<1>(p, G, lds, st);
    case 2: return launch_pipe_fmt<2>(p, G, lds, st);
    case 3: return launch_pipe_fmt<3>(p, G, lds, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pack_columns(const void *Rq, int64_t ldq_bytes, int fmt, const TileDesc *tiles, int n_valid,
                               int n_act, void *packed, int64_t ldp, hipStream_t st) {
  if (n_valid < 1 || ldp % 64 != 0 || ldp / 64 > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((2 * n_valid + 63) / 64), (unsigned)(ldp / 64));
  const int B = format_code_bytes(fmt);
  if (B == 4)
    pack_columns_kernel<uint32_t><<<grid, 256, 0, st>>>(static_cast<const uint32_t *>(Rq), ldq_bytes / 4, tiles,
                                                        n_valid, n_act, static_cast<uint32_t *>(packed), ldp);
  else if (B == 2)
    pack_columns_kernel<uint16_t><<<grid, 256, 0, st>>>(static_cast<const uint16_t *>(Rq), ldq_bytes / 2, tiles,
                                                        n_valid, n_act, static_cast<uint16_t *>(packed), ldp);
  else
    pack_columns_kernel<uint8_t><<<grid, 256, 0, st>>>(static_cast<const uint8_t *>(Rq), ldq_bytes, tiles, n_valid,
                                                       n_act, static_cast<uint8_t *>(packed), ldp);
  return hipGetLastError();
}

}  // namespace rtck
