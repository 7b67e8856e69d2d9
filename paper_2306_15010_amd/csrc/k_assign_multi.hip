// Fused nearest-codeword assignment (Alg. 1, Sec. 3.1) of several templates
// against one query map, for batched matching.
//
// Templates of equal padded codebook size are packed into passes of 8
// codeword blocks (128 codewords): a pass holds 8 templates of k <= 16, 4 of
// k <= 32, 2 of k <= 64 or one of k <= 128, their fragments concatenated per
// K-step.  One persistent launch walks the steps (tile, pass, group) with the
// refined kernel's pipeline (codebook group copied global->LDS one step
// ahead, query elements requested two steps ahead, one wait per step); the
// query tile is requested again for every pass, from L2 or the last-level
// cache after the first, so the map streams from HBM once while every
// template's codebook passes over it.  The epilogue of a pass works per
// template segment: its own top-2, error bound, label map and worklist, as
// the single-template refined kernel does for its one template.
#include "vqnnf_internal.h"
#include "dev_common.h"
#include "assign_common.h"
#include <type_traits>

namespace vqnnf {

constexpr int kMultiKB = 8;   // codeword blocks per pass

// The launch's tables (maps, passes, outputs) are written before the launch
// and only read by it: read through the constant address space, so that
// they come in as scalar loads (counted apart from the vector-memory
// requests in flight) instead of vector loads whose use would wait for the
// next tile's query and codebook requests as well.
template <typename T>
__device__ __forceinline__ T ld_const(const T* base, int64_t i) {
  static_assert(sizeof(T) % 4 == 0, "dword-sized table entries");
  const __attribute__((address_space(4))) uint32_t* w = (const __attribute__((address_space(4))) uint32_t*)(base + i);
  uint32_t d[sizeof(T) / 4];
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) d[k] = w[k];
  T v;
  __builtin_memcpy(&v, d, sizeof(T));
  return v;
}
static_assert(kWPB * 4 * 16 == kMultiTilePx, "tile of the fused launch");

// SG: the codebook fragments of block mb + 1 are read from LDS while the
// matrix cores work on block mb (as in the single-template refined kernel).
template <int NB, int QT, bool SG>
__global__ __launch_bounds__(kWPB * 64) void assign_multi_kernel(MultiParams p) {
  constexpr bool QF8 = QT == kQFP8;
  constexpr int KB = kMultiKB;
  constexpr int NT = kWPB * 64;
  constexpr int GF = 2 * KB * 64;                  // uint4 per load group (hi + lo)
  constexpr int CPT = GF / NT;                     // copies per thread per group
  constexpr int NEL = 8;                           // elements per lane per group
  constexpr int EB = QF8 ? 1 : 2;                  // bytes per query element
  constexpr int QW = NEL * EB / 4;                 // 32-bit words per lane per group
  constexpr int QN = NB;                           // vector loads per query request
  static_assert(GF % NT == 0, "whole copies");
  __shared__ uint4 st0[GF], st1[GF];
  __shared__ float cn_s[kMultiMaxPass * 16 * KB];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n = lane & 15, g = lane >> 4;
  const int ngr = p.n_groups;
  constexpr int TILE = kWPB * NB * 16;
  // a contiguous run of the launch's tiles per block
  const int64_t lo = p.n_tiles * blockIdx.x / gridDim.x;
  const int64_t hi = p.n_tiles * (blockIdx.x + 1) / gridDim.x;
  if (lo >= hi) return;

  // the map being processed (uniform per block)
  const char* mq = nullptr;
  int64_t mstride = 0, mpix = 0, mtiles = 0;
  __amdgpu_buffer_rsrc_t cb_rs;
  const MultiPass* mpasses = nullptr;
  const MultiOut* mouts = nullptr;
  int npass = 0;
  auto dma_cb = [&](int gs, uint4* stage) {   // global group index gs
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int base = i * NT + wave * 64;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(cb_rs, (lds_void_t*)(stage + base), 16, lane * 16,
                                               (gs * GF + base) * 16, 0, 0);
    }
  };
  uint32_t qoff[NB];
  // tile tl of the map; past the block's run it stands for tile `cur` (a
  // request that is never used but reads valid memory)
  auto set_tile = [&](int64_t tl, int64_t end, int64_t cur) {
    const int64_t t = tl < end ? tl : cur;
    const int64_t first = t * TILE;
    const int64_t lim = mpix - 1 - first;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      int64_t px = (int64_t)wave * NB * 16 + 16 * nb + n;
      px = px < lim ? px : lim;
      qoff[nb] = (uint32_t)(px * mstride * EB) + (uint32_t)(NEL * g * EB);
    }
    return mq + first * mstride * EB;
  };
  uint32_t qa[NB][QW], qb[NB][QW];
  auto load_q = [&](const char* tb, int gi, uint32_t (&dst)[NB][QW]) {
    const __amdgpu_buffer_rsrc_t rs = raw_rsrc(tb);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      if constexpr (QW == 2) {
        const uint2 v = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(rs, qoff[nb], gi * 32 * EB, 0));
        dst[nb][0] = v.x;
        dst[nb][QW - 1] = v.y;
      } else {
        const uint4 v = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, qoff[nb], gi * 32 * EB, 0));
        dst[nb][0] = v.x; dst[nb][1] = v.y; dst[nb][2] = v.z; dst[nb][QW - 1] = v.w;
      }
    }
  };

  f32x4_t acc[KB][NB];
  float qn2[NB];
  // a pass's accumulators start at ||c_j||^2 (one more addend of the FP32
  // sum, which the error bound counts), so the epilogue has nothing to add
  auto reset = [&](int pass) {
#pragma unroll
    for (int mb = 0; mb < KB; ++mb) {
      const f32x4_t c0 = *(const f32x4_t*)(cn_s + (pass * KB + mb) * 16 + 4 * g);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = c0;
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) qn2[nb] = 0.f;
  };
  auto compute = [&](const uint4* stage, uint32_t (&cur)[NB][QW]) {
    uint4 bq[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      if constexpr (QF8) {
        float x[8];
        fp8x8_to_f32(cur[nb][0], cur[nb][QW - 1], x);
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          qn2[nb] = fmaf(x[2 * i], x[2 * i], qn2[nb]);
          qn2[nb] = fmaf(x[2 * i + 1], x[2 * i + 1], qn2[nb]);
          w[i] = (__float_as_uint(x[2 * i]) >> 16) | (__float_as_uint(x[2 * i + 1]) & 0xFFFF0000u);
        }
        bq[nb] = make_uint4(w[0], w[1], w[2], w[3]);
      } else {
        const uint32_t ws[4] = {cur[nb][0], cur[nb][1], cur[nb][2], cur[nb][QW - 1]};
        bq[nb] = make_uint4(ws[0], ws[1], ws[2], ws[3]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float lo = __uint_as_float(ws[i] << 16), hi = __uint_as_float(ws[i] & 0xFFFF0000u);
          qn2[nb] = fmaf(lo, lo, qn2[nb]);
          qn2[nb] = fmaf(hi, hi, qn2[nb]);
        }
      }
    }
    // the query norm is the same for every pass of a tile; it is recomputed
    // each pass (the VALU work is small next to the products)
    if constexpr (SG) {
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
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = mfma_bf16(ah[mb & 1], bq[nb], acc[mb][nb]);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = mfma_bf16(al[mb & 1], bq[nb], acc[mb][nb]);
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
#pragma unroll
      for (int mb = 0; mb < KB; ++mb) {
        const uint4 ahi = stage[mb * 64 + lane];
        const uint4 alo = stage[(KB + mb) * 64 + lane];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          acc[mb][nb] = mfma_bf16(ahi, bq[nb], acc[mb][nb]);
          acc[mb][nb] = mfma_bf16(alo, bq[nb], acc[mb][nb]);
        }
      }
    }
  };

  // epilogue of one pass: templates of SB blocks each, in order from tmpl0
  auto finish_sb = [&](auto sb_tag, int64_t tile, int pass) {
    constexpr int SB = decltype(sb_tag)::value;
    constexpr int MW = (SB + 1) / 2;               // candidate mask words per template
    const MultiPass ps = ld_const(mpasses, pass);
    // upper bound of ||q|| per pixel block (shared by the pass's templates)
    float nqs[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      float q2 = qn2[nb];
      q2 += __uint_as_float(lane_xor16(__float_as_uint(q2), lane));
      q2 += __uint_as_float(lane_xor32(__float_as_uint(q2), lane));
      nqs[nb] = sqrtf(q2 * (1.0f + (float)(p.D + 8) * 0x1.0p-23f)) * (1.0f + 0x1.0p-20f);
    }
    // templates outer, pixel blocks inner: one table read per template
#pragma unroll
    for (int sg = 0; sg < KB / SB; ++sg) {
      if (sg >= ps.n_seg) break;
      const MultiOut o = ld_const(mouts, ps.tmpl0 + sg);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float nq = nqs[nb];
        const int64_t pix = tile * TILE + (int64_t)wave * NB * 16 + 16 * nb + n;
        const bool owner = (g == 0) && (pix < mpix);
        float v1 = 3.4e38f, v2 = 3.4e38f;
        int j1 = 0;
#pragma unroll
        for (int mb = sg * SB; mb < sg * SB + SB; ++mb)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float v = acc[mb][nb][i];
            const bool better = v < v1;
            v2 = __builtin_amdgcn_fmed3f(v1, v2, v);   // second best before the best moves
            j1 = better ? 16 * (mb - sg * SB) + i : j1;   // a constant operand; the lane's 4*g below
            v1 = better ? v : v1;                      // a select: no NaN canonicalisation
          }
        j1 += 4 * g;
#pragma unroll
        for (int m = 16; m <= 32; m <<= 1) {
          const float o1 = __uint_as_float(lane_xor(__float_as_uint(v1), m, lane));
          const float o2 = __uint_as_float(lane_xor(__float_as_uint(v2), m, lane));
          const int oj = (int)lane_xor((uint32_t)j1, m, lane);
          merge_top2_sel(v1, j1, v2, o1, oj, o2);
        }
        const float thr = (o.a0 + nq * (o.a1 + nq * o.a2)) * (1.0f + 0x1.0p-18f);
        const bool flagged = (v2 - v1) <= thr;
        if (owner) __builtin_amdgcn_raw_buffer_store_b8((uint8_t)j1, raw_rsrc(o.labels), (int)pix, 0, 0);
        const bool fl = owner && flagged;
        const unsigned long long bal = __ballot(fl);
        if (bal) {
          uint32_t mw[MW];
#pragma unroll
          for (int w = 0; w < MW; ++w) mw[w] = 0u;
#pragma unroll
          for (int mb = sg * SB; mb < sg * SB + SB; ++mb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int r = mb - sg * SB;
              if (acc[mb][nb][i] - v1 <= thr) mw[r >> 1] |= 1u << (16 * (r & 1) + 4 * g + i);
            }
#pragma unroll
          for (int w = 0; w < MW; ++w) {
            mw[w] |= lane_xor16(mw[w], lane);
            mw[w] |= lane_xor32(mw[w], lane);
          }
          uint32_t base = 0;
          if (lane == 0) base = atomicAdd(o.wl_count, (uint32_t)__popcll(bal));
          base = __builtin_amdgcn_readfirstlane(base);   // lane 0's: every lane is active here
          if (fl) {
            // resources based at the wave's first slot, offsets below 64 entries
            const uint32_t r = (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
            __builtin_amdgcn_raw_buffer_store_b32((uint32_t)pix, raw_rsrc(o.wl_pix + base), (int)(r * 4), 0, 0);
            const __amdgpu_buffer_rsrc_t wlm_rs = raw_rsrc(o.wl_mask + (size_t)base * MW);
#pragma unroll
            for (int w = 0; w < MW; ++w)
              __builtin_amdgcn_raw_buffer_store_b32(mw[w], wlm_rs, (int)((r * MW + w) * 4), 0, 0);
          }
        }
      }
    }
  };
  auto finish = [&](int64_t tile, int pass) {
    const int sb = ld_const(mpasses, pass).sb;
    if (sb == 8) finish_sb(std::integral_constant<int, 8>{}, tile, pass);
    else if (sb == 4) finish_sb(std::integral_constant<int, 4>{}, tile, pass);
    else if (sb == 2) finish_sb(std::integral_constant<int, 2>{}, tile, pass);
    else finish_sb(std::integral_constant<int, 1>{}, tile, pass);
  };

  // the map of the run's first tile
  int m = 0;
  for (int a = 0, b = p.n_maps - 1; a < b;) {
    const int c = (a + b + 1) / 2;
    if (ld_const(p.maps, c).tile0 <= lo) a = c, m = c; else b = c - 1;
  }
  for (int64_t t0 = lo; t0 < hi; ++m) {
    const MultiMap mm = ld_const(p.maps, m);
    mq = (const char*)mm.q;
    mstride = mm.stride;
    mpix = mm.n_pix;
    mtiles = multi_tiles(mpix);
    cb_rs = raw_rsrc(mm.frag);
    mpasses = mm.passes;
    mouts = mm.outs;
    npass = mm.n_pass;
    const int64_t first = t0 - mm.tile0, end = min(hi - mm.tile0, mtiles);
    const int nsteps = npass * ngr;                 // steps per tile
    // norms of the map's passes (the previous map's epilogues are done)
    __syncthreads();
    for (int i = threadIdx.x; i < npass * 16 * KB; i += NT) cn_s[i] = mm.cnorm[i];
    __syncthreads();   // the first pass's accumulators start from these norms
    const char* tb = set_tile(first, end, first);
    dma_cb(0, st0);
    load_q(tb, 0, qa);
    load_q(tb, 1, qb);
    wait_vm<0>();
    // groups per pass are even, so even steps use st0 and qa, odd steps st1 and qb
    for (int64_t tile = first; tile < end; ++tile) {
      const char* tb_next = tb;
      for (int pass = 0; pass < npass; ++pass) {
        reset(pass);
        for (int gi = 0; gi < ngr; gi += 2) {
          const int gs = pass * ngr + gi;            // global group of the even step
          const bool last_g = gi + 2 == ngr;         // last pair of the pass
          const bool last = last_g && pass + 1 == npass;
          {
            wait_vm<QN>();
            __syncthreads();
            dma_cb(gs + 1, st1);
            __builtin_amdgcn_sched_barrier(0);  // the copy stays ahead of later loads
            compute(st0, qa);
            if (last) tb_next = set_tile(tile + 1, end, tile);
            load_q(last ? tb_next : tb, last_g ? 0 : gi + 2, qa);
          }
          {
            wait_vm<QN>();
            __syncthreads();
            dma_cb(gs + 2 == nsteps ? 0 : gs + 2, st0);
            __builtin_amdgcn_sched_barrier(0);
            compute(st1, qb);
            if (last_g) finish(tile, pass);
            load_q(last ? tb_next : tb, last_g ? 1 : gi + 3, qb);
          }
        }
      }
      tb = tb_next;
    }
    // nothing of this map in flight when the next one starts
    wait_vm<0>();
    t0 = mm.tile0 + end;
  }
}

hipError_t launch_assign_multi(const MultiArgs& a, hipStream_t s, int n_cu) {
  const MultiParams& kp = a.kp;
  if (kp.n_maps < 1 || kp.n_tiles < 1 || kp.n_groups % 2 != 0) return hipErrorInvalidValue;
  const int grid = (int)std::min<int64_t>(kp.n_tiles, (int64_t)n_cu);
  // 1 (the default): the compiler's schedule; 2: fragments one block ahead
  // (measured about 2% slower on 64 templates of one 1024x1024 D=256 map)
  const bool sg = a.variant == 2;
  timing_begin(K_ASSIGN_MULTI);
  if (a.fp8) {
    if (sg) hipLaunchKernelGGL((assign_multi_kernel<4, kQFP8, true>), dim3(grid), dim3(kWPB * 64), 0, s, kp);
    else hipLaunchKernelGGL((assign_multi_kernel<4, kQFP8, false>), dim3(grid), dim3(kWPB * 64), 0, s, kp);
  } else {
    if (sg) hipLaunchKernelGGL((assign_multi_kernel<4, kQBF16, true>), dim3(grid), dim3(kWPB * 64), 0, s, kp);
    else hipLaunchKernelGGL((assign_multi_kernel<4, kQBF16, false>), dim3(grid), dim3(kWPB * 64), 0, s, kp);
  }
  timing_end(K_ASSIGN_MULTI);
  return hipGetLastError();
}

}  // namespace vqnnf
