// Persistent frames in the horizontal split of the paper's processing strategy
// (Section 2.2 and Figure 5): every workgroup calibrates its own subapertures
// and multiplies their slopes into its own columns of the control matrix --
// all actuator rows, kept on chip for the whole batch -- giving a partial
// actuator vector; the partial vectors are then added per actuator row by the
// row's owner (the tree vector addition of Section 2.3.5, done as a
// reduce-scatter across workgroups) and the integrator is applied.
//
// Design notes (MI355X / CDNA4):
//  * One workgroup of 256 threads (one wavefront per SIMD) per compute unit and
//    256 workgroups: thread t of every workgroup computes the rows of owner t,
//    so a producer's message to owner t is held by one thread and is written
//    with four-row device-coherent 16-byte stores, with no index arithmetic.
//  * Per thread the rows of its owner over the workgroup's 2 nch columns sit
//    in ordinary registers (RV rows), accumulation registers (RA rows, FP32
//    only) and LDS (the rest); at the ELT size nothing is read from memory but
//    the frame's pixels, the messages and the per-row scales.
//  * The frame's slopes never leave the workgroup: they go from the
//    calibration to LDS and from there to scalar registers, so the only
//    exchange between workgroups is the partial vectors, after the products.
//  * Owners read their messages with fully coalesced device-coherent 16-byte
//    loads (lane t reads piece t mod 8 of eight producers) and add them in a
//    fixed order: DPP across lane pairs, then LDS across rows and wavefronts,
//    so results are run-to-run deterministic.
#include "rtc_kernels.h"
#include "rtc_device.h"

namespace rtck {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int kBufWord3 = 0x00020000;   // buffer resource word 3 for raw dword access on gfx9
constexpr int kCoherent = 16;           // cache policy of a device-coherent access (sc1)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kBufWord3);
}

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Subapertures [kb, ke) of the workgroup, GS lanes per tile (one pixel row per
// lane), kHoriz / GS tiles a pass: slopes to sh_s (x of local subaperture kl at
// kl, y at nch + kl) and to the caller's optional per-frame arrays.  Rows are
// read as NPW 4-byte pixel pairs and 16-byte (dark, flat) pairs per lane (NPW
// = the widest tile's n / 2, rows of even width), all in flight before the
// first use; positions past a narrower row repeat its last pair.
template <int GS, int NPW>
__device__ __forceinline__ void horiz_calibration(const CalibArgs &a, int kb, int ke, int nch, const TileDesc *tl,
                                                  const float2 *rl, float *sh_s, int tid, int jz) {
  const int i = tid & (GS - 1);
  for (int k0 = kb; k0 < ke; k0 += kHoriz / GS) {
    const int kl = k0 - kb + tid / GS;
    const int k = kb + kl;
    const bool valid = k < ke;
    TileDesc t{};
    if (valid) t = tl[kl];
    const int n = t.n;
    const double half = 0.5 * (double)(n - 1);
    double S = 0.0, Sx = 0.0;
    int cnt = 0;
    if (valid && i < n) {
      const uint32_t *p2 = reinterpret_cast<const uint32_t *>(a.pix + (int64_t)t.off + (int64_t)i * t.pitch);
      const float4 *c2 = reinterpret_cast<const float4 *>(a.calib + (int64_t)t.calib_off + (int64_t)i * n);
      const int last = n / 2 - 1;
      uint32_t w[NPW];
      float4 c[NPW];
#pragma unroll
      for (int j = 0; j < NPW; ++j) {
        const int jj = j < last ? j : last;
        w[j] = p2[jj];
        c[j] = c2[jj];
      }
      uint32_t raw[2 * NPW];
      float2 cf[2 * NPW];
#pragma unroll
      for (int j = 0; j < NPW; ++j) {
        raw[2 * j] = w[j] & 0xffffu;
        raw[2 * j + 1] = w[j] >> 16;
        cf[2 * j] = make_float2(c[j].x, c[j].y);
        cf[2 * j + 1] = make_float2(c[j].z, c[j].w);
      }
      tile_row_sums<2 * NPW>(raw, cf, n, t.thr, a.mode, half, S, Sx, cnt, jz);
    }
    double cx, cy;
    tile_centroid<GS>(S, Sx, cnt, i, half, cx, cy, cnt);
    if (i == 0 && valid) {
      const float2 r = rl[kl];
      const float sx = (float)(cx - (double)r.x);
      const float sy = (float)(cy - (double)r.y);
      sh_s[kl] = sx;
      sh_s[nch + kl] = sy;
      if (a.s_user != nullptr) {
        a.s_user[t.sx] = sx;
        a.s_user[t.sy] = sy;
      }
      if (a.counts != nullptr) a.counts[k] = cnt;
    }
  }
}

// acc + one 16-byte chunk of codes times its EPC slope values, in column order.
template <int FMT>
__device__ __forceinline__ float chunk_fma(const uint4 &c, const float (&sq)[Codec<FMT>::EPC], float acc) {
  constexpr int EPC = Codec<FMT>::EPC;
  float v[EPC];
  Codec<FMT>::decode(c, v);
#pragma unroll
  for (int e = 0; e < EPC; ++e) acc = fmaf(v[e], sq[e], acc);
  return acc;
}

// Register tiers of a format and chunk count: RV row slots in ordinary
// registers, RA in accumulation registers, at most NT tail slots (LDS or
// memory); the row accumulators and one chunk of every tail slot are live
// while the products run.
template <int FMT, int NQ>
struct HShape {
  static constexpr int WORDS = NQ * 4;           // registers per row slot
  static constexpr int RV = FMT == 0 && NQ == 8 ? 5 : 128 / WORDS > 16 ? 16 : 128 / WORDS;
  static constexpr int RA = FMT == 0 && NQ == 8 ? 8 : 0;
};

// Chunk q of the NT tail row slots of thread tf from LDS (tail slot u at index
// u kHoriz + tf of the [NQ][lr] chunk array); branchless: the last slot of an
// owner with fewer rows reads a clamped (valid) index and is zeroed.
template <int NT, int RVA>
__device__ __forceinline__ void tail_chunks(uint4 (&t)[NT > 0 ? NT : 1], int q, int lr, int tf, int mr) {
  extern __shared__ uint4 lds[];
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    const int li = u * kHoriz + tf;
    const uint4 c = lds[q * lr + (li < lr ? li : lr - 1)];
    const bool ok = RVA + u < mr;
    t[u] = make_uint4(ok ? c.x : 0u, ok ? c.y : 0u, ok ? c.z : 0u, ok ? c.w : 0u);
  }
}

// FMT storage format, NQ 16-byte chunks per row slot (the workgroup's columns),
// NT tail row slots (every tail slot of the launch: rows past an owner's last
// read as zero), GS lanes per tile, NPW pixel pairs per lane row (4-byte pixel
// pairs only: tiles of even width on a 4-byte aligned frame); HShape gives the
// register tiers.  LDS: [NQ][lds_rows]
// chunks of the tail row slots, tail slot u of thread t at index u kHoriz + t
// (lds_rows = every tail row: the launcher refuses shapes that do not fit).
template <int FMT, int NQ, int NT, int GS, int NPW>
__global__ __launch_bounds__(kHoriz, 1) void horizontal_kernel(HorizArgs h, int32_t lds_rows) {
  constexpr int EPC = Codec<FMT>::EPC;
  constexpr int NC = NQ * EPC;                    // columns of a workgroup (padded)
  constexpr int RV = HShape<FMT, NQ>::RV, RA = HShape<FMT, NQ>::RA;
  constexpr int RVA = RV + RA;
  constexpr int PMAX = kHorizMsg / 4;             // four-row pieces of a message
  extern __shared__ uint4 lds[];
  __shared__ float sh_s[NC];
  __shared__ float4 sh_red[4][4][PMAX];            // [wavefront][row of 16 lanes][piece]
  __shared__ TileDesc sh_tiles[NC / 2];
  __shared__ float2 sh_ref[NC / 2];
  __shared__ uint32_t sh_abort, sh_bar;
  const PersistArgs &p = h.p;
  const MvmArgs &a = p.mvm;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int b = blockIdx.x;
  const int G = gridDim.x;                         // == kHoriz
  const int n_act = a.n_act;
  const int qrows = n_act / G, rem = n_act % G;
  const int my_rows = qrows + (tid < rem ? 1 : 0);     // rows of owner tid: this thread's row slots
  const int own_rows = qrows + (b < rem ? 1 : 0);      // rows this workgroup owns
  const int own_r0 = b * qrows + min(b, rem);
  const int kb = (int)(((int64_t)b * p.cal.n_valid) / G);
  const int ke = (int)(((int64_t)(b + 1) * p.cal.n_valid) / G);
  const int nch = h.nch;

  for (int k = kb + tid; k < ke; k += kHoriz) {
    const TileDesc t = p.cal.tiles[k];
    sh_tiles[k - kb] = t;
    sh_ref[k - kb] = make_float2(p.cal.ref[t.sx], p.cal.ref[t.sy]);
  }
  for (int j = tid; j < NC; j += kHoriz) sh_s[j] = 0.f;   // columns without a subaperture stay 0

  // the workgroup's columns of owner tid's rows: slots [0, RV) in registers,
  // [RV, RVA) in accumulation registers, the tail in LDS (or read each frame)
  const uint4 *hmb = h.hm + (int64_t)b * h.nrt * NQ * kHoriz;
  uint4 rv[RV > 0 ? RV : 1][NQ];
  uint4 ra[RA > 0 ? RA : 1][NQ];
#pragma unroll
  for (int i = 0; i < RV; ++i)
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      rv[i][q] = i < h.nrt ? hmb[((int64_t)i * NQ + q) * kHoriz + tid] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
  for (int i = 0; i < RA; ++i)
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      ra[i][q] = RV + i < h.nrt ? hmb[((int64_t)(RV + i) * NQ + q) * kHoriz + tid] : make_uint4(0u, 0u, 0u, 0u);
  for (int64_t c = tid; c < (int64_t)lds_rows * NQ; c += kHoriz) {
    const int q = (int)(c / lds_rows), li = (int)(c - (int64_t)q * lds_rows);
    const int u = li / kHoriz, t = li - u * kHoriz;
    lds[c] = hmb[((int64_t)(RVA + u) * NQ + q) * kHoriz + t];
  }
  float state = 0.f;
  if (tid < own_rows) state = a.state[own_r0 + tid];
  __syncthreads();

  const __amdgpu_buffer_rsrc_t xr = buffer_of(h.xbuf, (uint32_t)(2u * G * G * kHorizMsg * sizeof(float)));
  int frames_done = 0;
  for (int f = 0; f < p.n_frames; ++f) {
    // the register rows are loop-invariant codes: opaque per frame, so they are
    // decoded where used, and the RA rows stay in accumulation registers
#pragma unroll
    for (int i = 0; i < RV; ++i)
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        asm volatile("" : "+v"(rv[i][q].x), "+v"(rv[i][q].y), "+v"(rv[i][q].z), "+v"(rv[i][q].w));
#pragma unroll
    for (int i = 0; i < RA; ++i)
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        asm volatile("" : "+a"(ra[i][q].x), "+a"(ra[i][q].y), "+a"(ra[i][q].z), "+a"(ra[i][q].w));
    if (tid == 0) sh_abort = __hip_atomic_load(p.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (sh_abort) break;                            // a bounded wait expired somewhere: wind down
    if (p.ts != nullptr && b == 0 && tid == 0) p.ts[2 * f] = wall_clock64();
    trace_stamp(p, f, 0);
    // Per-frame opaque copies of the launch constants: without them the
    // compiler hoists every predicate, address and constant derived from them
    // out of the frame loop and holds it in registers for the whole batch.
    int tf = tid, mr = my_rows, jz = 0;
    asm volatile("" : "+v"(tf), "+v"(mr));
    int nrt = h.nrt, lr = lds_rows, kbf = kb, kef = ke, nchf = nch, orw = own_rows, orr = own_r0;
    asm volatile("" : "+s"(nrt), "+s"(lr), "+s"(kbf), "+s"(kef), "+s"(nchf), "+s"(orw), "+s"(orr), "+s"(jz));
    const int npcf = (nrt + 3) >> 2;

    // (a)-(b) this workgroup's subapertures: slopes into LDS
    CalibArgs ca = p.cal;
    ca.pix = p.cal.pix + (int64_t)f * p.frame_stride;
    ca.s_user = p.cal.s_user ? p.cal.s_user + (int64_t)f * 2 * p.cal.n_valid : nullptr;
    ca.counts = p.cal.counts ? p.cal.counts + (int64_t)f * p.cal.n_valid : nullptr;
    horiz_calibration<GS, NPW>(ca, kbf, kef, nchf, sh_tiles, sh_ref, sh_s, tf, jz);
    __syncthreads();
    trace_stamp(p, f, 1);

    // (c) the workgroup's columns times its slopes for owner tid's rows, one
    // column chunk at a time (its slopes in scalar registers): every row
    // accumulates in column order; the tail rows' chunks of a column chunk are
    // all loaded before the register rows' products of that chunk.
    float acc[RVA + NT];
#pragma unroll
    for (int i = 0; i < RVA + NT; ++i) acc[i] = 0.f;
    // tail chunks of column chunk q + 1 are loaded before the products of
    // chunk q; the accumulators are pinned after every chunk (a volatile asm
    // with a memory clobber), which keeps each chunk's products and loads in
    // place instead of letting the compiler batch all loads first
    uint4 tn[NT > 0 ? NT : 1];
    tail_chunks<NT, RVA>(tn, 0, lr, tf, mr);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      float sq[EPC];
#pragma unroll
      for (int e = 0; e < EPC; ++e)
        sq[e] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(sh_s[q * EPC + e])));
      uint4 tq[NT > 0 ? NT : 1];
#pragma unroll
      for (int u = 0; u < NT; ++u) tq[u] = tn[u];
      if (q + 1 < NQ) tail_chunks<NT, RVA>(tn, q + 1, lr, tf, mr);
#pragma unroll
      for (int i = 0; i < RV; ++i) acc[i] = chunk_fma<FMT>(rv[i][q], sq, acc[i]);
#pragma unroll
      for (int i = 0; i < RA; ++i) {
        uint4 m;
        asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(m.x) : "a"(ra[i][q].x));
        asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(m.y) : "a"(ra[i][q].y));
        asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(m.z) : "a"(ra[i][q].z));
        asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(m.w) : "a"(ra[i][q].w));
        acc[RV + i] = chunk_fma<FMT>(m, sq, acc[RV + i]);
      }
#pragma unroll
      for (int u = 0; u < NT; ++u) acc[RVA + u] = chunk_fma<FMT>(tq[u], sq, acc[RVA + u]);
#pragma unroll
      for (int i = 0; i < RVA + NT; ++i) asm volatile("" : "+v"(acc[i])::"memory");
    }
    // producer b's message to owner tid, four rows per 16-byte piece
    const int par = f & 1;
    const uint32_t msg = (uint32_t)(((par * G + tf) * G + b) * kHorizMsg) * (uint32_t)sizeof(float);
#pragma unroll
    for (int k = 0; k < (RVA + NT + 3) / 4; ++k) {
      if (4 * k < nrt) {
        float a4[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) a4[e] = 4 * k + e < RVA + NT ? acc[4 * k + e < RVA + NT ? 4 * k + e : 0] : 0.f;
        const v4f out = {a4[0], a4[1], a4[2], a4[3]};
        __builtin_amdgcn_raw_buffer_store_b128(out, xr, msg + 16u * (uint32_t)k, 0, kCoherent);
      }
    }
    trace_stamp(p, f, 4);
    // An expired wait leaves sh_bar set: the messages of frame f may then be
    // incomplete, so its commands and the rows' state are not written, and the
    // raised abort flag ends the loop at the next frame.
    (void)frame_barrier(p, (uint32_t)(f + 1), f, &sh_bar);
    trace_stamp(p, f, 2);
    if (p.ts != nullptr && f > 0 && wave == 0 && b == (f - 1) % G) reduce_end_stamp(p, f - 1);

    // (d) owner b: the G messages for its rows.  Lane t reads piece t mod 8 of
    // producers 32 j + t / 8 (coalesced: piece index j kHoriz + t), adds them
    // in j order, then lanes t and t + 8 of each row of 16 lanes are added.
    {
      const int pc = tf & 7;
      float4 s4 = make_float4(0.f, 0.f, 0.f, 0.f);
      const uint32_t base = (uint32_t)((par * G + b) * G * kHorizMsg) * (uint32_t)sizeof(float);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const v4f v = __builtin_amdgcn_raw_buffer_load_b128(xr, base + (uint32_t)(j * kHoriz + tf) * 16u, 0,
                                                             kCoherent);
        s4.x += v.x;
        s4.y += v.y;
        s4.z += v.z;
        s4.w += v.w;
      }
      s4.x += dpp_move<0x128>(s4.x);               // row_ror:8
      s4.y += dpp_move<0x128>(s4.y);
      s4.z += dpp_move<0x128>(s4.z);
      s4.w += dpp_move<0x128>(s4.w);
      if ((tf & 15) < 8 && pc < npcf) sh_red[tf >> 6][(tf >> 4) & 3][pc] = s4;
    }
    trace_stamp(p, f, 3);
    __syncthreads();
    if (tf < orw && (sh_bar & 1u) == 0u) {
      const float *red = reinterpret_cast<const float *>(sh_red);
      const int pc = tf >> 2, e = tf & 3;
      float v = 0.f;
#pragma unroll
      for (int w = 0; w < 4; ++w)
#pragma unroll
        for (int r = 0; r < 4; ++r) v += red[((w * 4 + r) * PMAX + pc) * 4 + e];
      const int row = orr + tf;
      if (a.scales != nullptr) v *= a.scales[row];
      float c = fmaf(a.gain, v, a.leak * state);
      c = fminf(fmaxf(c, a.cmd_min), a.cmd_max);
      state = c;
      a.cmd[(int64_t)f * n_act + row] = c;
      if (a.recon != nullptr) a.recon[(int64_t)f * n_act + row] = v;
    }
    trace_stamp(p, f, 5);
    if (p.ts != nullptr) {                         // this workgroup's commands of frame f are issued
      __syncthreads();
      if (tid == 0)
        __hip_atomic_store(reinterpret_cast<uint64_t *>(p.bar + sl::kEnds) + (f & 1) * sl::kMaxGroups + b,
                           wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    frames_done += (sh_bar & 1u) == 0u ? 1 : 0;
  }
  if (tid < own_rows) a.state[own_r0 + tid] = state;
  // end stamp of the last frame: the last workgroup to finish reduces it
  if (p.ts != nullptr && frames_done == p.n_frames) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (wave == 0) {
      int last = 0;
      if (tid == 0)
        last = __hip_atomic_fetch_add(p.bar + sl::kDone, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
               (uint32_t)G - 1;
      if (__builtin_amdgcn_readfirstlane(last)) reduce_end_stamp(p, p.n_frames - 1);
    }
  }
}

// Chunk (b, i, q, t) of the horizontal layout: the EB-byte codes of row
// rb(t) + i at columns [q EPC, (q + 1) EPC) of workgroup b (column j < nch:
// x slope of its subaperture kb + j, j < 2 nch: y slope of kb + j - nch);
// zero where the row or the subaperture does not exist.
template <int EB>
__global__ __launch_bounds__(256) void horiz_layout_kernel(const uint8_t *Rq, int64_t ldq_bytes,
                                                           const TileDesc *tiles, int n_valid, int n_act, int G,
                                                           int nch, int nrt, int nq, uint4 *hm) {
  constexpr int EPC = 16 / EB;
  const int64_t total = (int64_t)G * nrt * nq * kHoriz;
  const int qr = n_act / G, rm = n_act % G;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * 256) {
    const int t = (int)(idx % kHoriz);
    int64_t rest = idx / kHoriz;
    const int q = (int)(rest % nq);
    rest /= nq;
    const int i = (int)(rest % nrt);
    const int b = (int)(rest / nrt);
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    if (i < qr + (t < rm ? 1 : 0)) {
      const int64_t r = (int64_t)t * qr + min(t, rm) + i;
      const int kb = (int)(((int64_t)b * n_valid) / G), ke = (int)(((int64_t)(b + 1) * n_valid) / G);
      const uint8_t *row = Rq + r * ldq_bytes;
#pragma unroll
      for (int e = 0; e < EPC; ++e) {
        const int j = q * EPC + e;
        int pos = -1;
        if (j < nch) {
          if (kb + j < ke) pos = tiles[kb + j].sx;
        } else if (j < 2 * nch) {
          if (kb + j - nch < ke) pos = tiles[kb + j - nch].sy;
        }
        if (pos >= 0) {
          uint32_t code = 0;
          if constexpr (EB == 4) code = *reinterpret_cast<const uint32_t *>(row + (int64_t)pos * 4);
          if constexpr (EB == 2) code = *reinterpret_cast<const uint16_t *>(row + (int64_t)pos * 2);
          if constexpr (EB == 1) code = row[pos];
          w[(e * EB) / 4] |= code << (8 * ((e * EB) % 4));
        }
      }
    }
    hm[idx] = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

__global__ __launch_bounds__(256) void fill_zero_kernel(float *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0.f;
}

template <int FMT, int NQ, int NT, int GS, int NPW>
static hipError_t launch_horiz_variant(const HorizArgs &h, hipStream_t st) {
  using HS = HShape<FMT, NQ>;
  constexpr int RV = HS::RV, RA = HS::RA;
  if (h.nrt > RV + RA + NT) return hipErrorInvalidValue;
  auto kern = horizontal_kernel<FMT, NQ, NT, GS, NPW>;
  const int G = kHoriz;
  const int n_act = h.p.mvm.n_act;
  const int qrows = n_act / G, rem = n_act % G;
  const int64_t tail = qrows >= RV + RA ? (int64_t)(qrows - RV - RA) * kHoriz + rem : 0;
  int dev = 0, ncu = 0, lds_max = 0;
  hipError_t e;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess) return e;
  hipFuncAttributes fa{};
  if ((e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(kern))) != hipSuccess) return e;
  const int64_t avail = (int64_t)lds_max - (int64_t)fa.sharedSizeBytes;
  const int64_t cap = avail > 0 ? avail / (NQ * 16) : 0;
  if (tail > cap) return hipErrorInvalidValue;     // every row must stay on chip
  const int lds_rows = (int)tail;
  const size_t lds = (size_t)lds_rows * NQ * 16;
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds)) != hipSuccess)
    return e;
  int per_cu = 0;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kHoriz, lds)) != hipSuccess) return e;
  if (per_cu * ncu < G) return hipErrorCooperativeLaunchTooLarge;
  if ((e = launch_persist_reset(h.p.bar, h.p.abort_flag, G, st)) != hipSuccess) return e;
  HorizArgs ha = h;
  int32_t lr = lds_rows;
  void *args[] = {&ha, &lr};
  e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kern), dim3(G), dim3(kHoriz), args, lds, st);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

// Instantiated shapes: the tail-slot count of a launch is 0 (every row in
// registers) or NT1 (the ELT shapes: 5 FP32, 10 16-bit, 2 FP8 E4M3, 8 for the
// narrow column counts); NPW = 4 pixel pairs for tiles of up to 8 pixels,
// else 5 (FP32, up to 10 pixels: its registers hold the most rows) or 8.
template <int FMT, int NQ, int NT>
static hipError_t launch_horiz_nt(const HorizArgs &h, hipStream_t st) {
  constexpr bool WIDE_F32 = FMT == 0 && NQ == 8;
  const int n = h.p.cal.max_n;
  if (n <= 8) return launch_horiz_variant<FMT, NQ, NT, 8, 4>(h, st);
  if constexpr (WIDE_F32) {
    return n <= 10 ? launch_horiz_variant<FMT, NQ, NT, 16, 5>(h, st) : hipErrorInvalidValue;
  } else {
    return launch_horiz_variant<FMT, NQ, NT, 16, 8>(h, st);
  }
}
template <int FMT, int NQ, int NT1>
static hipError_t launch_horiz_gs(const HorizArgs &h, hipStream_t st) {
  const int tail = h.nrt - HShape<FMT, NQ>::RV - HShape<FMT, NQ>::RA;
  if (tail <= 0) return launch_horiz_nt<FMT, NQ, 0>(h, st);
  if (tail <= NT1) return launch_horiz_nt<FMT, NQ, NT1>(h, st);
  return hipErrorInvalidValue;
}

}  // namespace

int horiz_chunks(int fmt, int nch) {
  const int nc = 2 * nch;
  switch (fmt) {
    case 0: return nc <= 8 ? 2 : (nc <= 32 ? 8 : 0);
    case 1:
    case 2: return nc <= 8 ? 1 : (nc <= 32 ? 4 : 0);
    case 3: return nc <= 16 ? 1 : (nc <= 32 ? 2 : 0);
    default: return 0;
  }
}

int64_t horiz_layout_chunks(int G, int nrt, int nq) { return (int64_t)G * nrt * nq * kHoriz; }

int horiz_max_rows(int fmt, int nq) {
  switch (fmt * 16 + nq) {
    case 0 * 16 + 2: return HShape<0, 2>::RV + HShape<0, 2>::RA + 8;
    case 0 * 16 + 8: return HShape<0, 8>::RV + HShape<0, 8>::RA + 5;
    case 1 * 16 + 1: case 2 * 16 + 1: return HShape<1, 1>::RV + 8;
    case 1 * 16 + 4: case 2 * 16 + 4: return HShape<1, 4>::RV + 10;
    case 3 * 16 + 1: return HShape<3, 1>::RV + 8;
    case 3 * 16 + 2: return HShape<3, 2>::RV + 2;
    default: return 0;
  }
}

hipError_t launch_horiz_layout(const void *Rq, int64_t ldq_bytes, int fmt, const TileDesc *tiles, int n_valid,
                               int n_act, int G, int nch, int nrt, int nq, uint4 *hm, hipStream_t st) {
  const int64_t total = horiz_layout_chunks(G, nrt, nq);
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  const uint8_t *r = static_cast<const uint8_t *>(Rq);
  switch (fmt) {
    case 0:
      horiz_layout_kernel<4><<<(unsigned)blocks, 256, 0, st>>>(r, ldq_bytes, tiles, n_valid, n_act, G, nch, nrt, nq, hm);
      break;
    case 1:
    case 2:
      horiz_layout_kernel<2><<<(unsigned)blocks, 256, 0, st>>>(r, ldq_bytes, tiles, n_valid, n_act, G, nch, nrt, nq, hm);
      break;
    case 3:
      horiz_layout_kernel<1><<<(unsigned)blocks, 256, 0, st>>>(r, ldq_bytes, tiles, n_valid, n_act, G, nch, nrt, nq, hm);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fill_zero(float *p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  fill_zero_kernel<<<(unsigned)blocks, 256, 0, st>>>(p, n);
  return hipGetLastError();
}

hipError_t launch_horizontal(const HorizArgs &h, hipStream_t st) {
  if (h.p.n_frames <= 0) return hipSuccess;
  if (h.p.cal.max_n < 1 || h.p.cal.max_n > 16 || !h.p.cal.dark_fast || !h.p.vec) return hipErrorInvalidValue;
  if (h.nrt < 1 || h.nrt > kHorizMsg || h.p.mvm.n_act < 1) return hipErrorInvalidValue;
  const int nq = horiz_chunks(h.p.mvm.fmt, h.nch);
  switch (h.p.mvm.fmt) {
    case 0: return nq == 2 ? launch_horiz_gs<0, 2, 8>(h, st) : (nq == 8 ? launch_horiz_gs<0, 8, 5>(h, st) : hipErrorInvalidValue);
    case 1: return nq == 1 ? launch_horiz_gs<1, 1, 8>(h, st) : (nq == 4 ? launch_horiz_gs<1, 4, 10>(h, st) : hipErrorInvalidValue);
    case 2: return nq == 1 ? launch_horiz_gs<2, 1, 8>(h, st) : (nq == 4 ? launch_horiz_gs<2, 4, 10>(h, st) : hipErrorInvalidValue);
    case 3: return nq == 1 ? launch_horiz_gs<3, 1, 8>(h, st) : (nq == 2 ? launch_horiz_gs<3, 2, 2>(h, st) : hipErrorInvalidValue);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rtck
