// Nearest-codeword assignment (Alg. 1, Sec. 3.1) on gfx950 matrix cores.
//
// Distances are ranked by s_j = ||c_j||^2 - 2 q.c_j (the query norm is common
// to all codewords).  The contraction runs on MFMA with the codebook as the
// A operand (16 codewords per M block) and query pixels as the B operand (16
// pixels per N block); accumulators start at ||c_j||^2 and the codebook is
// pre-scaled by -2, so the accumulator ends at s_j.  The argmin is fused into
// the epilogue.
//
//  * FP32 plain path: v_mfma_f32_16x16x4_f32, argmin, no refinement.
//  * BF16 refined path: v_mfma_f32_16x16x32_bf16 with the codebook split into
//    BF16 hi + lo terms (FP32-stored queries split too: q_hi*c_hi +
//    q_hi*c_lo + q_lo*c_hi).  The epilogue keeps the best and second-best
//    score, evaluates the per-pixel error bound and appends every pixel whose
//    gap is inside it to a worklist, with the bit mask of codewords that are
//    still candidates.  The FP64 re-score kernel settles those pixels with the
//    exact sequential FP64 distance, lowest index on ties.
#include "vqnnf_internal.h"

#include <cstring>
#include "dev_common.h"
#include "assign_common.h"

namespace vqnnf {

// ------------------------------------------------------------------ timing
namespace {
thread_local TimingHook g_hook{nullptr, nullptr, nullptr};
const char* const kNames[K_COUNT] = {
    "fill",           "assign_fp32_plain", "assign_bf16_refined", "rescore_fp64",
    "integral_edges", "integral_prefix",   "integral_main",       "score_partial",
    "score_combine",  "score_integral", "assign_multi", "score_bank",
    "kmeans",         "assign_lowd",       "pca_project"};
}  // namespace

void set_timing_hook(const TimingHook* h) {
  if (h) g_hook = *h;
  else g_hook = TimingHook{nullptr, nullptr, nullptr};
}
void timing_begin(int id) {
  if (g_hook.begin) g_hook.begin(g_hook.user, id);
}
void timing_end(int id) {
  if (g_hook.end) g_hook.end(g_hook.user, id);
}
const char* kernel_name(int id) { return (id >= 0 && id < K_COUNT) ? kNames[id] : "?"; }

// ------------------------------------------------------------------ fill
__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  int blocks = (int)((n + 255) / 256);
  timing_begin(K_FILL);
  hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks), dim3(256), 0, s, p, v, n);
  timing_end(K_FILL);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, hipStream_t s) {
  return launch_fill_u32((uint32_t*)p, 0u, 2, s);
}

struct KParams {
  const void* q;
  int64_t stride;
  int64_t n_pix;
  int D;
  const void* frag;        // uint4 (bf16) or float (f32) fragments
  const float* cnorm;
  int n_groups;            // load groups along D
  int resident;            // whole codebook staged in LDS once
  int64_t n_tiles;
  uint8_t* labels;
  uint32_t* wl_count;
  uint32_t* wl_pix;
  uint32_t* wl_mask;
  float a0, a1, a2;
  float* dump;             // refined path, test support: s~_j to dump[pix * dump_stride + j]
  int dump_stride;
};

// Loads NE consecutive query elements of one pixel starting at element d0,
// zero beyond D.  QF32: values are floats; else BF16 bit patterns widened.
// VEC: 16-byte aligned rows; FULL: the caller guarantees d0 + NE <= D.
template <bool QF32, bool VEC, int NE, bool FULL = false>
__device__ __forceinline__ void load_query(const void* q, int64_t off, int d0, int D,
                                           uint32_t (&out)[QF32 ? NE : NE / 2]) {
  if (QF32) {
    const float* p = (const float*)q + off + d0;
    if (VEC && (FULL || d0 + NE <= D)) {
#pragma unroll
      for (int i = 0; i < NE / 4; ++i) {
        uint4 v = *(const uint4*)(p + 4 * i);
        out[4 * i] = v.x; out[4 * i + 1] = v.y; out[4 * i + 2] = v.z; out[4 * i + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int i = 0; i < NE; ++i) out[i] = (d0 + i < D) ? __float_as_uint(p[i]) : 0u;
    }
  } else {
    const uint16_t* p = (const uint16_t*)q + off + d0;
    if (VEC && (FULL || d0 + NE <= D)) {
      if (NE % 8 == 0) {
#pragma unroll
        for (int i = 0; i < NE / 8; ++i) {
          uint4 v = *(const uint4*)(p + 8 * i);
          out[4 * i] = v.x; out[4 * i + 1] = v.y; out[4 * i + 2] = v.z; out[4 * i + 3] = v.w;
        }
      } else {
#pragma unroll
        for (int i = 0; i < NE / 4; ++i) {
          uint2 v = *(const uint2*)(p + 4 * i);
          out[2 * i] = v.x; out[2 * i + 1] = v.y;
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < NE / 2; ++i) {
        uint32_t lo = (d0 + 2 * i < D) ? (uint32_t)p[2 * i] : 0u;
        uint32_t hi = (d0 + 2 * i + 1 < D) ? (uint32_t)p[2 * i + 1] : 0u;
        out[i] = lo | (hi << 16);
      }
    }
  }
}

// ============================================================ BF16 refined
// Template parameters: KB codeword blocks of 16, NB pixel blocks of 16 per
// wave, QF32: FP32-stored query (hi/lo split in registers), FAST: 16-byte
// aligned rows and D a multiple of 64 (every load group is full, no bounds
// checks).
//
// A block of 8 waves owns tiles of 8*NB*16 pixels and walks D in load groups
// of 32 elements (one K-step); the group count is even.  Work is a flat
// stream of (tile, group) steps.  Step s:
//   wait for the codebook group of step s to land in LDS, barrier;
//   start the direct global->LDS copy of group s+1 into the other stage (the
//   two stages are separate arrays, so the compiler can tell the stage being
//   filled from the one being read and adds no wait of its own);
//   multiply group s (codebook from LDS, query from registers);
//   at the end of a tile: epilogue (argmin, bound, worklist);
//   request the query elements of step s+2 into the register buffer just
//   consumed (two buffers: even and odd groups).
// Memory counters drain in issue order, so the wait for the codebook copy of
// step s leaves exactly the query loads of step s+1 outstanding.  With SG the
// codebook fragments of block mb+1 are read from LDS while the matrix cores
// work on block mb (the compiler otherwise reads each block just before its
// use and the LDS latency sits between the matrix-core groups).
struct StepCursor {
  int64_t tile;
  int gi;
};

template <int KB, int NB, int QT, bool FAST, bool SG>
__global__ __launch_bounds__(kWPB * 64) void assign_refined_kernel(KParams p) {
  constexpr bool QF32 = QT == kQF32, QF8 = QT == kQFP8;
  static_assert(!SG || !QF32, "fragments ahead: one query term");
  constexpr int NT = kWPB * 64;
  constexpr int GF = 2 * KB * 64;                  // uint4 per load group (hi + lo)
  constexpr int CPT = (GF + NT - 1) / NT;          // copies per thread per group
  constexpr int NEL = 8;                           // elements per lane per K-step
  constexpr int EB = QF32 ? 4 : QF8 ? 1 : 2;       // bytes per query element
  constexpr int QW = NEL * EB / 4;                 // 32-bit words per lane per K-step
  constexpr int QN = FAST ? NB * (QF32 ? 2 : 1) : 0;  // vector loads per query request
  constexpr int MW = (KB + 1) / 2;                 // candidate mask words
  // stages padded to whole copies (the padding receives duplicate data)
  __shared__ uint4 st0[CPT * NT], st1[CPT * NT];
  __shared__ float cn_s[16 * KB];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n = lane & 15, g = lane >> 4;
  const int ngr = p.n_groups;
  constexpr int TILE = kWPB * NB * 16;
  if ((int64_t)blockIdx.x >= p.n_tiles) return;

  auto advance = [&](StepCursor c) {
    if (++c.gi == ngr) {
      c.gi = 0;
      c.tile += gridDim.x;
    }
    return c;
  };
  // every wave copies its 1 KiB slices of the group; lane l writes 16 bytes
  // at slice + 16*l.  Issued unconditionally so that the memory counters
  // advance by the same amount on every path.
  const __amdgpu_buffer_rsrc_t cb_rs = raw_rsrc(p.frag);
  auto dma_cb = [&](int gi, uint4* stage) {
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int base = i * NT + wave * 64;
      const int sb = base < GF ? base : base % GF;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(cb_rs, (lds_void_t*)(stage + base), 16, lane * 16,
                                               (gi * GF + sb) * 16, 0, 0);
    }
  };
  // byte offset of this lane's pixel nb inside a tile, clamped to the last
  // pixel of the map (a past-the-end request reads valid memory and is never
  // used)
  uint32_t qoff[NB];
  auto set_tile = [&](int64_t tl) {
    const int64_t t = tl < p.n_tiles ? tl : (int64_t)blockIdx.x;
    const int64_t first = t * TILE;
    const int64_t lim = p.n_pix - 1 - first;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      int64_t px = (int64_t)wave * NB * 16 + 16 * nb + n;
      px = px < lim ? px : lim;
      qoff[nb] = (uint32_t)(px * p.stride * EB) + (uint32_t)(NEL * g * EB);
    }
    return (const char*)p.q + first * p.stride * EB;
  };
  uint32_t qa[NB][QW], qb[NB][QW];
  // query elements of K-step gi for the tile whose base set_tile returned
  auto load_q = [&](const char* tb, int gi, uint32_t (&dst)[NB][QW]) {
    if constexpr (FAST) {
      const __amdgpu_buffer_rsrc_t rs = raw_rsrc(tb);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        if constexpr (QW == 2) {
          const uint2 v = __builtin_bit_cast(
              uint2, __builtin_amdgcn_raw_buffer_load_b64(rs, qoff[nb], gi * 32 * EB, 0));
          dst[nb][0] = v.x;
          dst[nb][QW - 1] = v.y;
        } else {
#pragma unroll
          for (int i = 0; i < QW / 4; ++i) {
            const uint4 v = __builtin_bit_cast(
                uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, qoff[nb] + 16 * i, gi * 32 * EB, 0));
            dst[nb][4 * i] = v.x; dst[nb][4 * i + 1] = v.y;
            dst[nb][4 * i + 2] = v.z; dst[nb][4 * i + 3] = v.w;
          }
        }
      }
    } else if constexpr (QF8) {
      // byte loads with bounds checks, relative to the pixel row start
      const int d0 = gi * 32 + NEL * g;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const uint8_t* src = (const uint8_t*)tb + (qoff[nb] - (uint32_t)(NEL * g)) + d0;
        uint32_t w[2] = {0u, 0u};
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (d0 + i < p.D) w[i / 4] |= (uint32_t)src[i] << (8 * (i % 4));
        dst[nb][0] = w[0];
        dst[nb][QW - 1] = w[1];
      }
    } else {
      // element loads with bounds checks (D not a multiple of 64 or
      // unaligned rows), relative to the pixel row start
      const int d0 = gi * 32 + NEL * g;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int64_t row = (int64_t)(qoff[nb] - (uint32_t)(NEL * g * EB)) / EB;
        load_query<QF32, false, NEL>(tb, row, d0, p.D, dst[nb]);
      }
    }
  };
  // the codebook copy of the current step has landed once at most the query
  // loads of the next step are outstanding
  auto wait_stage = [&]() {
    if (QN > 0) wait_vm<QN>();
    else wait_vm<0>();
  };

  f32x4_t acc[KB][NB];
  float qn2[NB];
  auto reset = [&]() {  // new tile
#pragma unroll
    for (int mb = 0; mb < KB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) qn2[nb] = 0.f;
  };

  // multiply-accumulate of one group from an LDS stage and a query buffer
  auto compute = [&](const uint4* stage, uint32_t (&cur)[NB][QW]) {
    uint4 bhi[NB], blo[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      if constexpr (QF32) {
        uint32_t h[8], l[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float x = __uint_as_float(cur[nb][i]);
          qn2[nb] = fmaf(x, x, qn2[nb]);
          const uint32_t hb = f32_to_bf16_rne(x);
          const float r = x - bf16_bits_to_f32(hb);
          h[i] = hb;
          l[i] = f32_to_bf16_rne(r);
        }
        bhi[nb] = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16),
                             h[6] | (h[7] << 16));
        blo[nb] = make_uint4(l[0] | (l[1] << 16), l[2] | (l[3] << 16), l[4] | (l[5] << 16),
                             l[6] | (l[7] << 16));
      } else if constexpr (QF8) {
        // E4M3 codes are exact in BF16: the FP32 value's top half
        float x[8];
        fp8x8_to_f32(cur[nb][0], cur[nb][QW - 1], x);
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          qn2[nb] = fmaf(x[2 * i], x[2 * i], qn2[nb]);
          qn2[nb] = fmaf(x[2 * i + 1], x[2 * i + 1], qn2[nb]);
          w[i] = (__float_as_uint(x[2 * i]) >> 16) | (__float_as_uint(x[2 * i + 1]) & 0xFFFF0000u);
        }
        bhi[nb] = make_uint4(w[0], w[1], w[2], w[3]);
      } else {
        const uint32_t ws[4] = {cur[nb][0], cur[nb][1], cur[nb][2], cur[nb][3]};
        bhi[nb] = make_uint4(ws[0], ws[1], ws[2], ws[3]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float lo = __uint_as_float(ws[i] << 16), hi = __uint_as_float(ws[i] & 0xFFFF0000u);
          qn2[nb] = fmaf(lo, lo, qn2[nb]);
          qn2[nb] = fmaf(hi, hi, qn2[nb]);
        }
      }
    }
    if constexpr (SG) {
      // codebook fragments one block ahead: the LDS reads of block mb + 1
      // are in flight while the matrix cores work on block mb (the
      // scheduling barriers keep this order and both register sets live)
      uint4 ah[2], al[2];
      ah[0] = stage[lane];
      al[0] = stage[KB * 64 + lane];
#pragma unroll
      for (int mb = 0; mb < KB; ++mb) {
        if (mb + 1 < KB) {
          ah[(mb + 1) & 1] = stage[(mb + 1) * 64 + lane];
          al[(mb + 1) & 1] = stage[(KB + mb + 1) * 64 + lane];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = mfma_bf16(ah[mb & 1], bhi[nb], acc[mb][nb]);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = mfma_bf16(al[mb & 1], bhi[nb], acc[mb][nb]);
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
#pragma unroll
      for (int mb = 0; mb < KB; ++mb) {
        const uint4 ahi = stage[mb * 64 + lane];
        const uint4 alo = stage[(KB + mb) * 64 + lane];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          acc[mb][nb] = mfma_bf16(ahi, bhi[nb], acc[mb][nb]);
          acc[mb][nb] = mfma_bf16(alo, bhi[nb], acc[mb][nb]);
          if constexpr (QF32) acc[mb][nb] = mfma_bf16(ahi, blo[nb], acc[mb][nb]);
        }
      }
    }
  };

  // epilogue of a finished tile: s_j = ||c_j||^2 + (-2 q.c_j), the norm
  // added once after the products were accumulated from zero
  const __amdgpu_buffer_rsrc_t lab_rs = raw_rsrc(p.labels);
  auto finish = [&](int64_t tile) {
#pragma unroll
    for (int mb = 0; mb < KB; ++mb) {
      const f32x4_t c0 = *(const f32x4_t*)(cn_s + 16 * mb + 4 * g);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[mb][nb][i] = c0[i] + acc[mb][nb][i];
    }
    if (p.dump) {   // test support: the scores the bound is applied to
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int64_t pix = tile * TILE + (int64_t)wave * NB * 16 + 16 * nb + n;
        if (pix < p.n_pix)
#pragma unroll
          for (int mb = 0; mb < KB; ++mb)
            *(f32x4_t*)(p.dump + pix * p.dump_stride + 16 * mb + 4 * g) = acc[mb][nb];
      }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      // best (first index on ties) and second-best score of this lane's
      // codewords, in ascending index order, without branches: the second
      // best is the median of (best, second, new) before the best moves
      float v1 = 3.4e38f, v2 = 3.4e38f;
      int j1 = 0;
#pragma unroll
      for (int mb = 0; mb < KB; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float v = acc[mb][nb][i];
          const bool better = v < v1;
          v2 = __builtin_amdgcn_fmed3f(v1, v2, v);
          j1 = better ? 16 * mb + 4 * g + i : j1;
          v1 = better ? v : v1;
        }
      float q2 = qn2[nb];
      // merge over the four lane groups (lanes 16 and 32 apart)
#pragma unroll
      for (int m = 16; m <= 32; m <<= 1) {
        const float o1 = __uint_as_float(lane_xor(__float_as_uint(v1), m, lane));
        const float o2 = __uint_as_float(lane_xor(__float_as_uint(v2), m, lane));
        const int oj = (int)lane_xor((uint32_t)j1, m, lane);
        merge_top2_sel(v1, j1, v2, o1, oj, o2);
        q2 += __uint_as_float(lane_xor(__float_as_uint(q2), m, lane));
      }
      // upper bound of ||q||: FP32 sum of squares error, then sqrt rounding
      const float nq = sqrtf(q2 * (1.0f + (float)(p.D + 8) * 0x1.0p-23f)) * (1.0f + 0x1.0p-20f);
      const float thr = (p.a0 + nq * (p.a1 + nq * p.a2)) * (1.0f + 0x1.0p-18f);
      const bool flagged = (v2 - v1) <= thr;
      const int64_t pix = tile * TILE + (int64_t)wave * NB * 16 + 16 * nb + n;
      const bool owner = (g == 0) && (pix < p.n_pix);
      // stores through buffer resources: 32-bit offsets, scalar bases
      if (owner) __builtin_amdgcn_raw_buffer_store_b8((uint8_t)j1, lab_rs, (int)pix, 0, 0);
      const bool fl = owner && flagged;
      const unsigned long long bal = __ballot(fl);
      if (bal) {
        uint32_t mw[MW];
#pragma unroll
        for (int w = 0; w < MW; ++w) mw[w] = 0u;
#pragma unroll
        for (int mb = 0; mb < KB; ++mb)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (acc[mb][nb][i] - v1 <= thr) mw[mb >> 1] |= 1u << (16 * (mb & 1) + 4 * g + i);
#pragma unroll
        for (int w = 0; w < MW; ++w) {
          mw[w] |= lane_xor16(mw[w], lane);
          mw[w] |= lane_xor32(mw[w], lane);
        }
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(p.wl_count, (uint32_t)__popcll(bal));
        base = __builtin_amdgcn_readfirstlane(base);   // lane 0's: every lane is active here
        if (fl) {
          // resources based at the wave's first slot (64-bit pointer
          // arithmetic), so the 32-bit offsets stay below 64 entries
          const uint32_t r = (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
          __builtin_amdgcn_raw_buffer_store_b32((uint32_t)pix, raw_rsrc(p.wl_pix + base), (int)(r * 4), 0, 0);
          const __amdgpu_buffer_rsrc_t wlm_rs = raw_rsrc(p.wl_mask + (size_t)base * MW);
#pragma unroll
          for (int w = 0; w < MW; ++w)
            __builtin_amdgcn_raw_buffer_store_b32(mw[w], wlm_rs, (int)((r * MW + w) * 4), 0, 0);
        }
      }
    }
  };

  for (int i = threadIdx.x; i < 16 * KB; i += NT) cn_s[i] = p.cnorm[i];
  // one step: wait for its codebook group, barrier, start the copy of
  // group `fg` into `fill`, multiply group `cur` with `qbuf`
  auto step = [&](uint4* cur, uint4* fill, int fg, uint32_t (&qbuf)[NB][QW]) {
    wait_stage();
    __syncthreads();
    dma_cb(fg, fill);
    __builtin_amdgcn_sched_barrier(0);  // the copy stays ahead of later loads
    compute(cur, qbuf);
  };
  // prologue: group 0 of the first tile in stage st0, its query elements in
  // qa and those of group 1 in qb
  const char* tb = set_tile(blockIdx.x);
  dma_cb(0, st0);
  load_q(tb, 0, qa);
  load_q(tb, 1, qb);
  wait_vm<0>();
  // groups per tile are even, so even groups use stage st0 and buffer qa,
  // odd groups st1 and qb, across tiles too
  for (int64_t tile = blockIdx.x; tile < p.n_tiles; tile += gridDim.x) {
    reset();
    const char* tb_next = tb;
    for (int gi = 0; gi < ngr; gi += 2) {
      const bool last = gi + 2 == ngr;
      // even group gi; requests group gi + 2 (or group 0 of the next tile)
      step(st0, st1, gi + 1, qa);
      if (last) tb_next = set_tile(tile + gridDim.x);
      load_q(last ? tb_next : tb, last ? 0 : gi + 2, qa);
      // odd group gi + 1; requests group gi + 3 (or group 1 of the next tile)
      step(st1, st0, last ? 0 : gi + 2, qb);
      if (last) finish(tile);
      load_q(last ? tb_next : tb, last ? 1 : gi + 3, qb);
    }
    tb = tb_next;
  }
  // no copy into LDS may still be in flight when the workgroup retires
  wait_vm<0>();
}

// ============================================================ FP32 plain
// v_mfma_f32_16x16x4_f32: per K-step every lane supplies one element.  A load
// group is 4*E elements; lane group g reads elements [E*g, E*g + E) and K-step
// s of the group uses element E*g + s.  Same pipeline as the refined kernel:
// 8 waves, codebook groups double-buffered in LDS, query prefetched one group
// ahead, persistent blocks.
template <int KB, int NB, int E, int QT, bool VEC>
__global__ __launch_bounds__(kWPB * 64) void assign_plain_kernel(KParams p) {
  constexpr bool QF32 = QT == kQF32, QF8 = QT == kQFP8;
  extern __shared__ float4 ldsf[];
  constexpr int NT = kWPB * 64;
  constexpr int GF = E * KB * 64 / 4;              // float4 per load group
  constexpr int CPT = (GF + NT - 1) / NT;
  constexpr int QW = QF32 ? E : QF8 ? (E + 3) / 4 : E / 2;   // 32-bit words per lane per group
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int n = lane & 15, g = lane >> 4;
  const float4* frag = (const float4*)p.frag;
  const int ngr = p.n_groups;
  constexpr int64_t TILE = kWPB * NB * 16;
  int64_t tile = blockIdx.x;
  if (tile >= p.n_tiles) return;

  auto pix_off = [&](int64_t tl, int nb) {
    int64_t pix = tl * TILE + (int64_t)wave * NB * 16 + 16 * nb + n;
    if (pix >= p.n_pix) pix = p.n_pix - 1;
    return pix * p.stride;
  };
  float4 cbr[CPT];
  uint32_t cur[NB][QW], nxt[NB][QW];
  auto load_cb = [&](int gi) {
    const float4* src = frag + (int64_t)gi * GF;
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int idx = threadIdx.x + i * NT;
      if (idx < GF) cbr[i] = src[idx];
    }
  };
  auto load_q = [&](int64_t tl, int gi, uint32_t (&dst)[NB][QW]) {
    const int d0 = gi * 4 * E + E * g;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      if constexpr (QF8) {
        // E codes of one pixel (element 0 in the low byte)
        const uint8_t* src = (const uint8_t*)p.q + pix_off(tl, nb) + d0;
        if (VEC && d0 + E <= p.D) {
          if constexpr (E == 8) {
            const uint2 v = *(const uint2*)src;
            dst[nb][0] = v.x;
            dst[nb][QW - 1] = v.y;
          } else {
            dst[nb][0] = *(const uint32_t*)src;
          }
        } else {
#pragma unroll
          for (int w = 0; w < QW; ++w) dst[nb][w] = 0u;
#pragma unroll
          for (int i = 0; i < E; ++i)
            if (d0 + i < p.D) dst[nb][i / 4] |= (uint32_t)src[i] << (8 * (i % 4));
        }
      } else {
        load_query<QF32, VEC, E>(p.q, pix_off(tl, nb), d0, p.D, dst[nb]);
      }
    }
  };
  load_cb(0);
  load_q(tile, 0, cur);
  int buf = 0;
  for (;;) {
    f32x4_t acc[KB][NB];
#pragma unroll
    for (int mb = 0; mb < KB; ++mb)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    for (int gi = 0; gi < ngr; ++gi) {
      float4* stage4 = ldsf + buf * GF;
#pragma unroll
      for (int i = 0; i < CPT; ++i) {
        const int idx = threadIdx.x + i * NT;
        if (idx < GF) stage4[idx] = cbr[i];
      }
      __syncthreads();
      const bool more_g = gi + 1 < ngr;
      const int64_t ntile = more_g ? tile : tile + gridDim.x;
      const int ngi = more_g ? gi + 1 : 0;
      const bool have_next = ntile < p.n_tiles;
      if (have_next) {
        load_cb(ngi);
        load_q(ntile, ngi, nxt);
      }
      const float* stage = (const float*)stage4;
      float x[NB][E];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        if constexpr (QF32) {
#pragma unroll
          for (int i = 0; i < E; ++i) x[nb][i] = __uint_as_float(cur[nb][i]);
        } else if constexpr (QF8) {
#pragma unroll
          for (int w = 0; w < E / 4; ++w) {
            const f32x2_t lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)cur[nb][w], false);
            const f32x2_t hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)cur[nb][w], true);
            x[nb][4 * w] = lo[0];
            x[nb][4 * w + 1] = lo[1];
            x[nb][4 * w + 2] = hi[0];
            x[nb][4 * w + 3] = hi[1];
          }
        } else {
#pragma unroll
          for (int i = 0; i < E / 2; ++i) {
            x[nb][2 * i] = __uint_as_float(cur[nb][i] << 16);
            x[nb][2 * i + 1] = __uint_as_float(cur[nb][i] & 0xFFFF0000u);
          }
        }
      }
#pragma unroll
      for (int s = 0; s < E; ++s)
#pragma unroll
        for (int mb = 0; mb < KB; ++mb) {
          const float a = stage[(s * KB + mb) * 64 + lane];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, x[nb][s], acc[mb][nb], 0, 0, 0);
        }
      buf ^= 1;
      if (have_next) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int i = 0; i < QW; ++i) cur[nb][i] = nxt[nb][i];
      }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      float v1 = 3.4e38f;
      int j1 = 0;
#pragma unroll
      for (int mb = 0; mb < KB; ++mb) {
        const f32x4_t c0 = *(const f32x4_t*)(p.cnorm + 16 * mb + 4 * g);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float v = c0[i] + acc[mb][nb][i];
          if (v < v1) { v1 = v; j1 = 16 * mb + 4 * g + i; }
        }
      }
#pragma unroll
      for (int m = 16; m <= 32; m <<= 1) {
        const float o = __shfl_xor(v1, m);
        const int oj = __shfl_xor(j1, m);
        if (o < v1 || (o == v1 && oj < j1)) { v1 = o; j1 = oj; }
      }
      const int64_t pix = tile * TILE + (int64_t)wave * NB * 16 + 16 * nb + n;
      if (g == 0 && pix < p.n_pix) p.labels[pix] = (uint8_t)j1;
    }
    tile += gridDim.x;
    if (tile >= p.n_tiles) break;
  }
}

// ============================================================ FP64 re-score
// Pixels flagged by the refined kernel are settled with the distance
// d_j = sum_t (q_t - c_j,t)^2, sequential in t from 0 with separate FP64
// subtract, multiply and add, for every candidate j of the pixel's mask; the
// smallest d wins, the lowest index on ties.
//
// A wave takes kRPix worklist pixels.  Their (pixel, candidate) pairs are
// numbered in pixel order with candidates ascending and dealt to the lanes 64
// at a time, one sequential sum per lane; the query and codeword elements of
// the next kRPF steps of kRStep elements are requested while the current ones
// are summed.  After each round the lane of pixel s merges that round's
// results of pixel s in pair order.
struct RParams {
  const void* q;
  int64_t stride;
  int D, k, mask_words;
  const float* codebook;
  const float* scale;      // FP8 maps: [D] channel scales
  const uint32_t* wl_count;
  const uint32_t* wl_pix;
  const uint32_t* wl_mask;
  uint8_t* labels;
  int img_w, img_h;          // RGB images: colour features are built from pixels
};

constexpr int kRPix = 32;    // worklist pixels per wave
constexpr int kRStep = 8;    // elements per load step
constexpr int kRPF = 4;      // steps per prefetch block

// Query element t as the FP64 value the oracle uses: FP32, BF16, or an
// E4M3FN code times its channel scale (exact in FP64).
template <int QT>
__device__ __forceinline__ double q_elem(const void* q, int64_t off, int t, const float* scale) {
  if constexpr (QT == kQF32) return (double)((const float*)q)[off + t];
  else if constexpr (QT == kQFP8) {
    const f32x2_t v = __builtin_amdgcn_cvt_pk_f32_fp8((int)((const uint8_t*)q)[off + t], false);
    return (double)v[0] * (double)scale[t];
  } else {
    return (double)bf16_bits_to_f32(((const uint16_t*)q)[off + t]);
  }
}

// Candidate j < k of a mask word w.
__device__ __forceinline__ uint32_t valid_bits(uint32_t bits, int w, int k) {
  const int lim = k - 32 * w;
  return lim <= 0 ? 0u : (lim >= 32 ? bits : bits & ((1u << lim) - 1u));
}

__device__ __forceinline__ int nth_candidate(const uint32_t* m, int mw, int k, uint32_t r) {
  for (int w = 0; w < mw; ++w) {
    uint32_t bits = valid_bits(m[w], w, k);
    const uint32_t n = (uint32_t)__popc(bits);
    if (r < n) {
      for (; r > 0; --r) bits &= bits - 1u;
      return 32 * w + __ffs(bits) - 1;
    }
    r -= n;
  }
  return -1;
}

// Sequential FP64 distance of one query row to one codeword row.  VEC: both
// rows 16-byte aligned; steps of kRStep elements, then a scalar tail.
template <int QT, bool VEC>
__device__ double seq_dist(const void* q, int64_t qoff, const float* c, int D, const float* scale) {
#pragma clang fp contract(off)
  constexpr bool QF32 = QT == kQF32, QF8 = QT == kQFP8;
  constexpr int QV = QF32 ? 2 : 1;   // uint4 per step of the query row (FP8: one uint2)
  constexpr int SV = QF8 ? 2 : 1;    // uint4 of scales per step
  double acc = 0.0;
  const int nst = VEC ? D / kRStep : 0;
  if (nst > 0) {
    const char* qb8 = (const char*)q + qoff * (QF32 ? 4 : QF8 ? 1 : 2);
    const uint4* qp = (const uint4*)qb8;
    const uint2* qp8 = (const uint2*)qb8;
    const uint4* cp = (const uint4*)c;
    const uint4* sp = (const uint4*)scale;
    uint4 qa[kRPF][QV], ca[kRPF][2], qb[kRPF][QV], cb[kRPF][2];
    uint4 sa[kRPF][SV], sb[kRPF][SV];
    // requests of a block are clamped to the last step: always in bounds
    auto load_blk = [&](int s0, uint4 (&qd)[kRPF][QV], uint4 (&cd)[kRPF][2], uint4 (&sd)[kRPF][SV]) {
#pragma unroll
      for (int i = 0; i < kRPF; ++i) {
        const int st = min(s0 + i, nst - 1);
        if constexpr (QF8) {
          const uint2 v = qp8[st];
          qd[i][0] = make_uint4(v.x, v.y, 0u, 0u);
          sd[i][0] = sp[st * 2];
          sd[i][SV - 1] = sp[st * 2 + 1];
        } else {
#pragma unroll
          for (int v = 0; v < QV; ++v) qd[i][v] = qp[st * QV + v];
        }
        cd[i][0] = cp[st * 2];
        cd[i][1] = cp[st * 2 + 1];
      }
    };
    auto sum_blk = [&](int s0, const uint4 (&qd)[kRPF][QV], const uint4 (&cd)[kRPF][2],
                       const uint4 (&sd)[kRPF][SV]) {
#pragma unroll
      for (int i = 0; i < kRPF; ++i) {
        if (s0 + i >= nst) break;
        const uint32_t cw[8] = {cd[i][0].x, cd[i][0].y, cd[i][0].z, cd[i][0].w,
                                cd[i][1].x, cd[i][1].y, cd[i][1].z, cd[i][1].w};
        double qv[8];
        if constexpr (QF32) {
          const uint32_t qw[8] = {qd[i][0].x, qd[i][0].y, qd[i][0].z, qd[i][0].w,
                                  qd[i][QV - 1].x, qd[i][QV - 1].y, qd[i][QV - 1].z, qd[i][QV - 1].w};
#pragma unroll
          for (int e = 0; e < 8; ++e) qv[e] = (double)__uint_as_float(qw[e]);
        } else if constexpr (QF8) {
          float x[8];
          fp8x8_to_f32(qd[i][0].x, qd[i][0].y, x);
          const uint32_t sw[8] = {sd[i][0].x, sd[i][0].y, sd[i][0].z, sd[i][0].w,
                                  sd[i][SV - 1].x, sd[i][SV - 1].y, sd[i][SV - 1].z, sd[i][SV - 1].w};
#pragma unroll
          for (int e = 0; e < 8; ++e) qv[e] = (double)x[e] * (double)__uint_as_float(sw[e]);
        } else {
          const uint32_t ws[4] = {qd[i][0].x, qd[i][0].y, qd[i][0].z, qd[i][0].w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            qv[2 * e] = (double)__uint_as_float(ws[e] << 16);
            qv[2 * e + 1] = (double)__uint_as_float(ws[e] & 0xFFFF0000u);
          }
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const double dq = qv[e] - (double)__uint_as_float(cw[e]);
          const double sq = dq * dq;
          acc = acc + sq;
        }
      }
    };
    load_blk(0, qa, ca, sa);
    for (int s0 = 0; s0 < nst; s0 += 2 * kRPF) {
      load_blk(s0 + kRPF, qb, cb, sb);
      sum_blk(s0, qa, ca, sa);
      load_blk(s0 + 2 * kRPF, qa, ca, sa);
      sum_blk(s0 + kRPF, qb, cb, sb);
    }
  }
  for (int t = nst * kRStep; t < D; ++t) {
    const double dq = q_elem<QT>(q, qoff, t, scale) - (double)c[t];
    const double sq = dq * dq;
    acc = acc + sq;
  }
  return acc;
}

// The same sequential FP64 distance for a colour feature of an RGB image:
// element t = (3*dy + dx)*3 + c is channel c of the pixel at (x + dx - 1,
// y + dy - 1), edges replicated (D = 27).
__device__ double seq_dist_rgb(const RParams& p, uint32_t pix, const float* c) {
#pragma clang fp contract(off)
  const uint8_t* img = (const uint8_t*)p.q;
  const int y = (int)(pix / (uint32_t)p.img_w), x = (int)(pix - (uint32_t)y * (uint32_t)p.img_w);
  double acc = 0.0;
  for (int t = 0; t < 27; ++t) {
    const int dy = t / 9, dx = (t / 3) % 3, ch = t % 3;
    const int yy = min(max(y + dy - 1, 0), p.img_h - 1), xx = min(max(x + dx - 1, 0), p.img_w - 1);
    const double dq = (double)img[((int64_t)yy * p.img_w + xx) * p.stride + ch] - (double)c[t];
    const double sq = dq * dq;
    acc = acc + sq;
  }
  return acc;
}

// Block `blk` of `nblk` walks the worklist of one (template, map) pair.
template <int QT, bool VEC>
__device__ __forceinline__ void rescore_body(const RParams& p, uint32_t blk, uint32_t nblk) {
  __shared__ uint32_t pfx[kRPix + 1];   // exclusive prefix of candidate counts
  __shared__ double rd[64];
  __shared__ int rj[64];
  const int lane = threadIdx.x;
  const int mw = p.mask_words;
  const uint32_t count = *p.wl_count;
  for (uint32_t g0 = blk * kRPix; g0 < count; g0 += nblk * kRPix) {
    const uint32_t npx = min((uint32_t)kRPix, count - g0);
    uint32_t nc = 0;
    if (lane < (int)npx) {
      const uint32_t* m = p.wl_mask + (int64_t)(g0 + lane) * mw;
      for (int w = 0; w < mw; ++w) nc += (uint32_t)__popc(valid_bits(m[w], w, p.k));
    }
    const uint32_t inc = wave_incl_scan(nc);
    const uint32_t total = (uint32_t)__shfl((int)inc, 63);
    if (lane < kRPix) pfx[lane] = inc - nc;
    if (lane == 0) pfx[kRPix] = total;
    __syncthreads();
    double best = 0.0;   // lane s < npx: running best of pixel s
    int bj = -1;
    for (uint32_t P0 = 0; P0 < total; P0 += 64) {
      const uint32_t P = P0 + lane;
      double d = 0.0;
      int j = -1;
      if (P < total) {
        int s = 0;   // last slot with pfx[s] <= P: the pixel owning pair P
#pragma unroll
        for (int step = kRPix / 2; step >= 1; step >>= 1)
          if (pfx[s + step] <= P) s += step;
        j = nth_candidate(p.wl_mask + (int64_t)(g0 + s) * mw, mw, p.k, P - pfx[s]);
        if constexpr (QT == kQRGB8) {
          d = seq_dist_rgb(p, p.wl_pix[g0 + s], p.codebook + (int64_t)j * p.D);
        } else {
          const int64_t qoff = (int64_t)p.wl_pix[g0 + s] * p.stride;
          d = seq_dist<QT, VEC>(p.q, qoff, p.codebook + (int64_t)j * p.D, p.D, p.scale);
        }
      }
      rd[lane] = d;
      rj[lane] = j;
      __syncthreads();
      if (lane < (int)npx) {
        const uint32_t a = max(pfx[lane], P0), b = min(pfx[lane + 1], P0 + 64);
        for (uint32_t r = a; r < b; ++r) {
          const double dd = rd[r - P0];
          if (bj < 0 || dd < best) {
            best = dd;
            bj = rj[r - P0];
          }
        }
      }
      __syncthreads();
    }
    if (lane < (int)npx && bj >= 0) p.labels[p.wl_pix[g0 + lane]] = (uint8_t)bj;
    __syncthreads();
  }
}

template <int QT, bool VEC>
__global__ __launch_bounds__(64) void rescore_kernel(RParams p) {
  rescore_body<QT, VEC>(p, blockIdx.x, gridDim.x);
}

// Batched: blockIdx.y selects the pair.
template <int QT, bool VEC>
__global__ __launch_bounds__(64) void rescore_batch_kernel(const RParams* __restrict__ tab) {
  rescore_body<QT, VEC>(tab[blockIdx.y], blockIdx.x, gridDim.x);
}

// ============================================================ launchers
namespace {

// Query rows start `align`-byte aligned (base and pixel stride).
bool rows_aligned(const AssignArgs& a, int elem_bytes, int align) {
  uintptr_t base = (uintptr_t)a.q;
  return (base % align == 0) && ((a.stride * elem_bytes) % align == 0);
}

int qtype(int dtype) { return dtype == VQNNF_F32 ? kQF32 : dtype == VQNNF_FP8_E4M3 ? kQFP8 : kQBF16; }
int qbytes(int qt) { return qt == kQF32 ? 4 : qt == kQFP8 ? 1 : 2; }

template <int KB, int NB, int QT, bool FAST, bool SG>
hipError_t go_refined(const KParams& kp, int grid, hipStream_t s) {
  hipLaunchKernelGGL((assign_refined_kernel<KB, NB, QT, FAST, SG>), dim3(grid), dim3(kWPB * 64), 0, s, kp);
  return hipGetLastError();
}

template <int KB, int NB, int QT>
hipError_t go_refined_f(const KParams& kp, int grid, bool fast, int var, hipStream_t s) {
  if (!fast) return go_refined<KB, NB, QT, false, false>(kp, grid, s);
  if constexpr (QT != kQF32 && KB <= 8)
    if (var == 2) return go_refined<KB, NB, QT, true, true>(kp, grid, s);
  return go_refined<KB, NB, QT, true, false>(kp, grid, s);
}

template <int KB, int NB>
hipError_t go_refined_q(const KParams& kp, int grid, int qt, bool fast, int var, hipStream_t s) {
  if (qt == kQF32) return go_refined_f<KB, NB, kQF32>(kp, grid, fast, var, s);
  if (qt == kQFP8) return go_refined_f<KB, NB, kQFP8>(kp, grid, fast, var, s);
  return go_refined_f<KB, NB, kQBF16>(kp, grid, fast, var, s);
}

template <int KB, int NB, int E, int QT, bool VEC>
hipError_t go_plain(const KParams& kp, size_t lds, int grid, hipStream_t s) {
  auto kern = assign_plain_kernel<KB, NB, E, QT, VEC>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kWPB * 64), lds, s, kp);
  return hipGetLastError();
}

template <int KB, int NB, int QT>
hipError_t go_plain_e(const KParams& kp, size_t lds, int grid, int E, bool vec, hipStream_t s) {
  if (E == 8) return vec ? go_plain<KB, NB, 8, QT, true>(kp, lds, grid, s)
                         : go_plain<KB, NB, 8, QT, false>(kp, lds, grid, s);
  return vec ? go_plain<KB, NB, 4, QT, true>(kp, lds, grid, s)
             : go_plain<KB, NB, 4, QT, false>(kp, lds, grid, s);
}

template <int KB, int NB>
hipError_t go_plain_s(const KParams& kp, size_t lds, int grid, int E, int qt, bool vec, hipStream_t s) {
  if (qt == kQF32) return go_plain_e<KB, NB, kQF32>(kp, lds, grid, E, vec, s);
  if (qt == kQFP8) return go_plain_e<KB, NB, kQFP8>(kp, lds, grid, E, vec, s);
  return go_plain_e<KB, NB, kQBF16>(kp, lds, grid, E, vec, s);
}

template <int QT>
hipError_t go_rescore(const RParams& rp, int grid, bool vec, hipStream_t s) {
  if (vec) hipLaunchKernelGGL((rescore_kernel<QT, true>), dim3(grid), dim3(64), 0, s, rp);
  else hipLaunchKernelGGL((rescore_kernel<QT, false>), dim3(grid), dim3(64), 0, s, rp);
  return hipGetLastError();
}

template <int QT>
hipError_t go_rescore_b(const RParams* tab, int grid, int n, bool vec, hipStream_t s) {
  if (vec) hipLaunchKernelGGL((rescore_batch_kernel<QT, true>), dim3(grid, n), dim3(64), 0, s, tab);
  else hipLaunchKernelGGL((rescore_batch_kernel<QT, false>), dim3(grid, n), dim3(64), 0, s, tab);
  return hipGetLastError();
}

RParams make_rparams(const AssignArgs& a) {
  const DeviceTemplate& t = *a.t;
  RParams rp{};
  rp.q = a.q;
  rp.stride = a.stride;
  rp.D = a.D;
  rp.k = t.k;
  rp.mask_words = a.mask_words > 0 ? a.mask_words : (t.geom.kpad + 31) / 32;
  rp.codebook = t.d_codebook;
  rp.scale = a.scale;
  rp.wl_count = a.wl_count;
  rp.wl_pix = a.wl_pix;
  rp.wl_mask = a.wl_mask;
  rp.labels = a.labels;
  rp.img_w = a.img_w;
  rp.img_h = a.img_h;
  return rp;
}

// whole steps of 8 elements: query rows aligned to the step width (16 bytes;
// 8 for FP8 codes) and codeword rows 16-byte aligned
bool rescore_vec(const AssignArgs& a) {
  const int qt = qtype(a.dtype);
  return a.dtype != VQNNF_RGB8 && rows_aligned(a, qbytes(qt), qt == kQFP8 ? 8 : 16) && (a.D % 4 == 0);
}

}  // namespace

// Pixel blocks per wave: KB*NB*4 accumulators stay <= 128 registers.
static int pick_nb(int kb) { return kb <= 8 ? 4 : 2; }

// Schedule of the refined kernel: 1 the compiler's, 2 codebook fragments
// read one block ahead of the matrix cores.  Variant 2 exists for aligned
// BF16 / FP8 rows with at most 128 codewords and is their default
// (a.variant 0); other maps always take variant 1.
int refined_variants(const AssignArgs& a) {
  const AssignGeom& g = a.t->geom;
  const int qt = qtype(a.dtype);
  const bool fast = rows_aligned(a, qbytes(qt), qt == kQFP8 ? 8 : 16) && (a.D % 64 == 0) && g.s_bf16 == 1;
  return (fast && qt != kQF32 && g.kb <= 8) ? 2 : 1;
}
static int refined_variant(const AssignArgs& a) {
  const int n = refined_variants(a);
  if (a.variant >= 1 && a.variant <= n) return a.variant;
  return n;
}

hipError_t launch_assign_refined(const AssignArgs& a, hipStream_t s, int n_cu) {
  const DeviceTemplate& t = *a.t;
  const AssignGeom& g = t.geom;
  KParams kp{};
  kp.q = a.q;
  kp.stride = a.stride;
  kp.n_pix = a.n_pix;
  kp.D = a.D;
  kp.frag = a.frag_bf16;
  kp.cnorm = t.d_cnorm;
  kp.n_groups = g.d_pad_bf16 / (32 * g.s_bf16);
  kp.labels = a.labels;
  kp.wl_count = a.wl_count;
  kp.wl_pix = a.wl_pix;
  kp.wl_mask = a.wl_mask;
  kp.a0 = a.bound.a0;
  kp.a1 = a.bound.a1;
  kp.a2 = a.bound.a2;
  kp.dump = a.dump;
  kp.dump_stride = g.kpad;
  const int qt = qtype(a.dtype);
  // full load groups: D a multiple of two K-steps of 32, rows aligned to the
  // query load width (16 bytes; 8 for FP8 codes)
  const bool fast = rows_aligned(a, qbytes(qt), qt == kQFP8 ? 8 : 16) && (a.D % 64 == 0) &&
                    g.s_bf16 == 1;
  const int NB = pick_nb(g.kb);
  const int64_t tile_px = (int64_t)kWPB * NB * 16;
  kp.n_tiles = (a.n_pix + tile_px - 1) / tile_px;
  const int grid = (int)std::min<int64_t>(kp.n_tiles, (int64_t)n_cu);
  if (g.s_bf16 != 1 || kp.n_groups % 2 != 0) return hipErrorInvalidValue;
  const int var = refined_variant(a);
  timing_begin(K_ASSIGN_REFINED);
  hipError_t e;
  switch (g.kb) {
    case 1: e = go_refined_q<1, 4>(kp, grid, qt, fast, var, s); break;
    case 2: e = go_refined_q<2, 4>(kp, grid, qt, fast, var, s); break;
    case 3: e = go_refined_q<3, 4>(kp, grid, qt, fast, var, s); break;
    case 4: e = go_refined_q<4, 4>(kp, grid, qt, fast, var, s); break;
    case 8: e = go_refined_q<8, 4>(kp, grid, qt, fast, var, s); break;
    case 16: e = go_refined_q<16, 2>(kp, grid, qt, fast, var, s); break;
    default: e = hipErrorInvalidValue; break;
  }
  timing_end(K_ASSIGN_REFINED);
  return e;
}

hipError_t launch_assign_plain(const AssignArgs& a, hipStream_t s, int n_cu) {
  const DeviceTemplate& t = *a.t;
  const AssignGeom& g = t.geom;
  KParams kp{};
  kp.q = a.q;
  kp.stride = a.stride;
  kp.n_pix = a.n_pix;
  kp.D = a.D;
  kp.frag = a.frag_f32;
  kp.cnorm = t.d_cnorm;
  kp.n_groups = g.d_pad_f32 / (4 * g.e_f32);
  kp.labels = a.labels;
  const int qt = qtype(a.dtype);
  const bool vec = rows_aligned(a, qbytes(qt), qt == kQFP8 ? 8 : 16);
  const size_t lds = 2 * (size_t)g.e_f32 * g.kb * 64 * 4;
  const int NB = pick_nb(g.kb);
  const int64_t tile_px = (int64_t)kWPB * NB * 16;
  kp.n_tiles = (a.n_pix + tile_px - 1) / tile_px;
  const int grid = (int)std::min<int64_t>(kp.n_tiles, (int64_t)n_cu);
  timing_begin(K_ASSIGN_PLAIN);
  hipError_t e;
  const int E = g.e_f32;
  switch (g.kb) {
    case 1: e = go_plain_s<1, 4>(kp, lds, grid, E, qt, vec, s); break;
    case 2: e = go_plain_s<2, 4>(kp, lds, grid, E, qt, vec, s); break;
    case 3: e = go_plain_s<3, 4>(kp, lds, grid, E, qt, vec, s); break;
    case 4: e = go_plain_s<4, 4>(kp, lds, grid, E, qt, vec, s); break;
    case 8: e = go_plain_s<8, 4>(kp, lds, grid, E, qt, vec, s); break;
    case 16: e = go_plain_s<16, 2>(kp, lds, grid, E, qt, vec, s); break;
    default: e = hipErrorInvalidValue; break;
  }
  timing_end(K_ASSIGN_PLAIN);
  return e;
}

hipError_t launch_rescore(const AssignArgs& a, hipStream_t s, int n_cu) {
  const RParams rp = make_rparams(a);
  const int qt = qtype(a.dtype);
  const bool vec = rescore_vec(a);
  const int grid = n_cu * 4;   // one wave per block; waves stride over the worklist
  timing_begin(K_RESCORE);
  hipError_t e;
  if (a.dtype == VQNNF_RGB8) e = go_rescore<kQRGB8>(rp, grid, false, s);
  else if (qt == kQF32) e = go_rescore<kQF32>(rp, grid, vec, s);
  else if (qt == kQFP8) e = go_rescore<kQFP8>(rp, grid, vec, s);
  else e = go_rescore<kQBF16>(rp, grid, vec, s);
  timing_end(K_RESCORE);
  return e;
}

void plan_rescore_batch(const std::vector<AssignArgs>& pairs, RescoreBatchPlan* out) {
  out->blob.clear();
  out->launches.clear();
  for (int cls = 0; cls < 8; ++cls) {   // (query type, vector path)
    std::vector<RParams> tab;
    for (const AssignArgs& a : pairs) {
      const int qt = a.dtype == VQNNF_RGB8 ? kQRGB8 : qtype(a.dtype);
      if (qt * 2 + (rescore_vec(a) ? 1 : 0) == cls) tab.push_back(make_rparams(a));
    }
    if (tab.empty()) continue;
    const size_t off = (out->blob.size() + 63) / 64 * 64;
    out->blob.resize(off + tab.size() * sizeof(RParams));
    std::memcpy(out->blob.data() + off, tab.data(), tab.size() * sizeof(RParams));
    out->launches.push_back({cls / 2, cls % 2, off, (int)tab.size()});
  }
}

hipError_t launch_rescore_batch(const RescoreBatchPlan& pl, const uint8_t* d_blob, int n_cu, hipStream_t s) {
  for (const RescoreBatchPlan::Launch& l : pl.launches) {
    const RParams* tab = (const RParams*)(d_blob + l.tab_off);
    const int grid = n_cu;   // per pair; waves stride over its worklist
    timing_begin(K_RESCORE);
    hipError_t e;
    if (l.qt == kQRGB8) e = go_rescore_b<kQRGB8>(tab, grid, l.n, false, s);
    else if (l.qt == kQF32) e = go_rescore_b<kQF32>(tab, grid, l.n, l.vec != 0, s);
    else if (l.qt == kQFP8) e = go_rescore_b<kQFP8>(tab, grid, l.n, l.vec != 0, s);
    else e = go_rescore_b<kQBF16>(tab, grid, l.n, l.vec != 0, s);
    timing_end(K_RESCORE);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
}  // namespace vqnnf
