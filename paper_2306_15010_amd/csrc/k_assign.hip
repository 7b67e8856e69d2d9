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

namespace vqnnf {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ timing
namespace {
thread_local TimingHook g_hook{nullptr, nullptr, nullptr};
const char* const kNames[K_COUNT] = {
    "fill",           "assign_fp32_plain", "assign_bf16_refined", "rescore_fp64",
    "integral_edges", "integral_prefix",   "integral_main",       "score_fused",
    "score_integral"};
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

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ float bf16_bits_to_f32(uint32_t b) { return __uint_as_float(b << 16); }

__device__ __forceinline__ uint32_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
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
};

// Loads NE consecutive query elements of one pixel starting at element d0,
// zero beyond D.  QF32: values are floats; else BF16 bit patterns widened.
template <bool QF32, bool VEC, int NE>
__device__ __forceinline__ void load_query(const void* q, int64_t off, int d0, int D,
                                           uint32_t (&out)[QF32 ? NE : NE / 2]) {
  if (QF32) {
    const float* p = (const float*)q + off + d0;
    if (VEC && d0 + NE <= D) {
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
    if (VEC && d0 + NE <= D) {
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

__device__ __forceinline__ f32x4_t mfma_bf16(uint4 a, uint4 b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                 __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
}

// Top-2 merge of (best value, best index, second value) triples; ties in the
// best value keep the lower index and make the second equal to the best.
__device__ __forceinline__ void merge_top2(float& v1, int& j1, float& v2, float o1, int oj1,
                                           float o2) {
  if (o1 < v1 || (o1 == v1 && oj1 < j1)) {
    v2 = fminf(v1, o2);
    v1 = o1;
    j1 = oj1;
  } else {
    v2 = fminf(v2, o1);
  }
}

// ============================================================ BF16 refined
// Template parameters: KB codeword blocks of 16, NB pixel blocks of 16 per
// wave, S K-steps (of 32 elements) per load group, QF32: FP32-stored query
// (hi/lo split in registers), VEC: 16-byte aligned rows, WPB waves per block.
template <int KB, int NB, int S, bool QF32, bool VEC, int WPB>
__global__ __launch_bounds__(WPB * 64) void assign_refined_kernel(KParams p) {
  extern __shared__ uint4 lds[];
  constexpr int GROUP_FRAGS = S * 2 * KB * 64;     // uint4 per load group
  constexpr int NEL = 8 * S;                       // elements per lane per group
  constexpr int MW = (KB + 1) / 2;                 // candidate mask words
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int n = lane & 15, g = lane >> 4;
  const uint4* frag = (const uint4*)p.frag;

  if (p.resident) {
    const int total = p.n_groups * GROUP_FRAGS;
    for (int i = threadIdx.x; i < total; i += WPB * 64) lds[i] = frag[i];
    __syncthreads();
  }

  for (int64_t tile = blockIdx.x; tile < p.n_tiles; tile += gridDim.x) {
    const int64_t pix0 = tile * (WPB * NB * 16) + (int64_t)wave * NB * 16;
    f32x4_t acc[KB][NB];
#pragma unroll
    for (int mb = 0; mb < KB; ++mb) {
      f32x4_t c0 = *(const f32x4_t*)(p.cnorm + 16 * mb + 4 * g);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = c0;
    }
    float qn2[NB];
    int64_t off[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      qn2[nb] = 0.f;
      int64_t pix = pix0 + 16 * nb + n;
      if (pix >= p.n_pix) pix = p.n_pix - 1;
      off[nb] = pix * p.stride;
    }

    for (int gi = 0; gi < p.n_groups; ++gi) {
      const uint4* a_src;
      if (!p.resident) {
        __syncthreads();
        const uint4* src = frag + (int64_t)gi * GROUP_FRAGS;
        for (int i = threadIdx.x; i < GROUP_FRAGS; i += WPB * 64) lds[i] = src[i];
        __syncthreads();
        a_src = lds;
      } else {
        a_src = lds + gi * GROUP_FRAGS;
      }
      const int d0 = gi * 32 * S + NEL * g;
      uint32_t qraw[NB][QF32 ? NEL : NEL / 2];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) load_query<QF32, VEC, NEL>(p.q, off[nb], d0, p.D, qraw[nb]);

#pragma unroll
      for (int s = 0; s < S; ++s) {
        uint4 bhi[NB], blo[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          if (QF32) {
            uint32_t h[8], l[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              float x = __uint_as_float(qraw[nb][8 * s + i]);
              qn2[nb] = fmaf(x, x, qn2[nb]);
              uint32_t hb = f32_to_bf16_rne(x);
              float r = x - bf16_bits_to_f32(hb);
              h[i] = hb;
              l[i] = f32_to_bf16_rne(r);
            }
            bhi[nb] = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16),
                                 h[6] | (h[7] << 16));
            blo[nb] = make_uint4(l[0] | (l[1] << 16), l[2] | (l[3] << 16), l[4] | (l[5] << 16),
                                 l[6] | (l[7] << 16));
          } else {
            uint32_t w0 = qraw[nb][4 * s], w1 = qraw[nb][4 * s + 1];
            uint32_t w2 = qraw[nb][4 * s + 2], w3 = qraw[nb][4 * s + 3];
            bhi[nb] = make_uint4(w0, w1, w2, w3);
            uint32_t ws[4] = {w0, w1, w2, w3};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              float lo = __uint_as_float(ws[i] << 16), hi = __uint_as_float(ws[i] & 0xFFFF0000u);
              qn2[nb] = fmaf(lo, lo, qn2[nb]);
              qn2[nb] = fmaf(hi, hi, qn2[nb]);
            }
          }
        }
#pragma unroll
        for (int mb = 0; mb < KB; ++mb) {
          const uint4 ahi = a_src[((s * 2 + 0) * KB + mb) * 64 + lane];
          const uint4 alo = a_src[((s * 2 + 1) * KB + mb) * 64 + lane];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) {
            acc[mb][nb] = mfma_bf16(ahi, bhi[nb], acc[mb][nb]);
            acc[mb][nb] = mfma_bf16(alo, bhi[nb], acc[mb][nb]);
            if (QF32) acc[mb][nb] = mfma_bf16(ahi, blo[nb], acc[mb][nb]);
          }
        }
      }
    }

    // ---------------------------------------------------------- epilogue
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      float v1 = 3.4e38f, v2 = 3.4e38f;
      int j1 = 0;
#pragma unroll
      for (int mb = 0; mb < KB; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float v = acc[mb][nb][i];
          int j = 16 * mb + 4 * g + i;
          if (v < v1) { v2 = v1; v1 = v; j1 = j; }
          else if (v < v2) { v2 = v; }
        }
      float q2 = qn2[nb];
#pragma unroll
      for (int m = 16; m <= 32; m <<= 1) {
        float o1 = __shfl_xor(v1, m), o2 = __shfl_xor(v2, m);
        int oj = __shfl_xor(j1, m);
        merge_top2(v1, j1, v2, o1, oj, o2);
        q2 += __shfl_xor(q2, m);
      }
      // upper bound of ||q||: FP32 sum of squares error, then sqrt rounding
      float nq = sqrtf(q2 * (1.0f + (float)(p.D + 8) * 0x1.0p-23f)) * (1.0f + 0x1.0p-20f);
      float thr = (p.a0 + nq * (p.a1 + nq * p.a2)) * (1.0f + 0x1.0p-18f);
      bool flagged = (v2 - v1) <= thr;
      const int64_t pix = pix0 + 16 * nb + n;
      const bool owner = (g == 0) && (pix < p.n_pix);
      if (owner) p.labels[pix] = (uint8_t)j1;
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
          mw[w] |= __shfl_xor(mw[w], 16);
          mw[w] |= __shfl_xor(mw[w], 32);
        }
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(p.wl_count, (uint32_t)__popcll(bal));
        base = __shfl(base, 0);
        if (fl) {
          uint32_t slot = base + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
          p.wl_pix[slot] = (uint32_t)pix;
#pragma unroll
          for (int w = 0; w < MW; ++w) p.wl_mask[(int64_t)slot * MW + w] = mw[w];
        }
      }
    }
  }
}

// ============================================================ FP32 plain
// v_mfma_f32_16x16x4_f32: per K-step every lane supplies one element.  A load
// group is 4*E elements; lane group g reads elements [E*g, E*g + E) and K-step
// s of the group uses element E*g + s.
template <int KB, int NB, int E, bool QF32, bool VEC, int WPB>
__global__ __launch_bounds__(WPB * 64) void assign_plain_kernel(KParams p) {
  extern __shared__ float ldsf[];
  constexpr int GROUP = E * KB * 64;   // floats per load group
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int n = lane & 15, g = lane >> 4;
  const float* frag = (const float*)p.frag;

  if (p.resident) {
    const int total = p.n_groups * GROUP;
    for (int i = threadIdx.x; i < total; i += WPB * 64) ldsf[i] = frag[i];
    __syncthreads();
  }
  for (int64_t tile = blockIdx.x; tile < p.n_tiles; tile += gridDim.x) {
    const int64_t pix0 = tile * (WPB * NB * 16) + (int64_t)wave * NB * 16;
    f32x4_t acc[KB][NB];
#pragma unroll
    for (int mb = 0; mb < KB; ++mb) {
      f32x4_t c0 = *(const f32x4_t*)(p.cnorm + 16 * mb + 4 * g);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = c0;
    }
    int64_t off[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      int64_t pix = pix0 + 16 * nb + n;
      if (pix >= p.n_pix) pix = p.n_pix - 1;
      off[nb] = pix * p.stride;
    }
    for (int gi = 0; gi < p.n_groups; ++gi) {
      const float* a_src;
      if (!p.resident) {
        __syncthreads();
        const float* src = frag + (int64_t)gi * GROUP;
        for (int i = threadIdx.x; i < GROUP; i += WPB * 64) ldsf[i] = src[i];
        __syncthreads();
        a_src = ldsf;
      } else {
        a_src = ldsf + gi * GROUP;
      }
      const int d0 = gi * 4 * E + E * g;
      float x[NB][E];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        if (QF32) {
          uint32_t r[E];
          load_query<true, VEC, E>(p.q, off[nb], d0, p.D, r);
#pragma unroll
          for (int i = 0; i < E; ++i) x[nb][i] = __uint_as_float(r[i]);
        } else {
          uint32_t r[E / 2];
          load_query<false, VEC, E>(p.q, off[nb], d0, p.D, r);
#pragma unroll
          for (int i = 0; i < E / 2; ++i) {
            x[nb][2 * i] = __uint_as_float(r[i] << 16);
            x[nb][2 * i + 1] = __uint_as_float(r[i] & 0xFFFF0000u);
          }
        }
      }
#pragma unroll
      for (int s = 0; s < E; ++s)
#pragma unroll
        for (int mb = 0; mb < KB; ++mb) {
          const float a = a_src[(s * KB + mb) * 64 + lane];
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, x[nb][s], acc[mb][nb], 0, 0, 0);
        }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      float v1 = 3.4e38f;
      int j1 = 0;
#pragma unroll
      for (int mb = 0; mb < KB; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float v = acc[mb][nb][i];
          if (v < v1) { v1 = v; j1 = 16 * mb + 4 * g + i; }
        }
#pragma unroll
      for (int m = 16; m <= 32; m <<= 1) {
        float o = __shfl_xor(v1, m);
        int oj = __shfl_xor(j1, m);
        if (o < v1 || (o == v1 && oj < j1)) { v1 = o; j1 = oj; }
      }
      const int64_t pix = pix0 + 16 * nb + n;
      if (g == 0 && pix < p.n_pix) p.labels[pix] = (uint8_t)j1;
    }
  }
}

// ============================================================ FP64 re-score
// One thread per flagged pixel: FP64 distances to every candidate codeword in
// the fixed order d = sum_t (q_t - c_t)^2, sequential in t from 0, separate
// subtract, multiply and add; strict < over ascending indices keeps the
// lowest index on ties.
struct RParams {
  const void* q;
  int64_t stride;
  int D, k, mask_words, qf32;
  const float* codebook;
  const uint32_t* wl_count;
  const uint32_t* wl_pix;
  const uint32_t* wl_mask;
  uint8_t* labels;
};

__global__ __launch_bounds__(256) void rescore_kernel(RParams p) {
#pragma clang fp contract(off)
  const uint32_t count = *p.wl_count;
  for (uint32_t it = blockIdx.x * blockDim.x + threadIdx.x; it < count;
       it += gridDim.x * blockDim.x) {
    const uint32_t pix = p.wl_pix[it];
    const uint32_t* mask = p.wl_mask + (int64_t)it * p.mask_words;
    double best = 0.0;
    int bj = -1;
    for (int w = 0; w < p.mask_words; ++w) {
      uint32_t bits = mask[w];
      while (bits) {
        int b = __ffs(bits) - 1;
        bits &= bits - 1u;
        int j = 32 * w + b;
        if (j >= p.k) continue;
        const float* c = p.codebook + (int64_t)j * p.D;
        double acc = 0.0;
        if (p.qf32) {
          const float* q = (const float*)p.q + (int64_t)pix * p.stride;
          for (int t = 0; t < p.D; ++t) {
            double d = (double)q[t] - (double)c[t];
            double sq = d * d;
            acc = acc + sq;
          }
        } else {
          const uint16_t* q = (const uint16_t*)p.q + (int64_t)pix * p.stride;
          for (int t = 0; t < p.D; ++t) {
            double d = (double)bf16_bits_to_f32(q[t]) - (double)c[t];
            double sq = d * d;
            acc = acc + sq;
          }
        }
        if (bj < 0 || acc < best) { best = acc; bj = j; }
      }
    }
    if (bj >= 0) p.labels[pix] = (uint8_t)bj;
  }
}

// ============================================================ launchers
namespace {

bool rows_aligned(const AssignArgs& a, int elem_bytes) {
  uintptr_t base = (uintptr_t)a.q;
  return (base % 16 == 0) && ((a.stride * elem_bytes) % 16 == 0);
}

template <int KB, int NB, int S, bool QF32, bool VEC, int WPB>
hipError_t go_refined(const KParams& kp, size_t lds, int grid, hipStream_t s) {
  auto kern = assign_refined_kernel<KB, NB, S, QF32, VEC, WPB>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(WPB * 64), lds, s, kp);
  return hipGetLastError();
}

template <int KB, int NB, int S, bool QF32, int WPB>
hipError_t go_refined_v(const KParams& kp, size_t lds, int grid, bool vec, hipStream_t s) {
  return vec ? go_refined<KB, NB, S, QF32, true, WPB>(kp, lds, grid, s)
             : go_refined<KB, NB, S, QF32, false, WPB>(kp, lds, grid, s);
}

template <int KB, int NB, int WPB>
hipError_t go_refined_s(const KParams& kp, size_t lds, int grid, int S, bool qf32, bool vec,
                        hipStream_t s) {
  if (qf32) {
    if (S == 4) return go_refined_v<KB, NB, 4, true, WPB>(kp, lds, grid, vec, s);
    if (S == 2) return go_refined_v<KB, NB, 2, true, WPB>(kp, lds, grid, vec, s);
    return go_refined_v<KB, NB, 1, true, WPB>(kp, lds, grid, vec, s);
  }
  if (S == 4) return go_refined_v<KB, NB, 4, false, WPB>(kp, lds, grid, vec, s);
  if (S == 2) return go_refined_v<KB, NB, 2, false, WPB>(kp, lds, grid, vec, s);
  return go_refined_v<KB, NB, 1, false, WPB>(kp, lds, grid, vec, s);
}

template <int KB, int NB, int E, bool QF32, bool VEC, int WPB>
hipError_t go_plain(const KParams& kp, size_t lds, int grid, hipStream_t s) {
  auto kern = assign_plain_kernel<KB, NB, E, QF32, VEC, WPB>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(WPB * 64), lds, s, kp);
  return hipGetLastError();
}

template <int KB, int NB, int WPB>
hipError_t go_plain_s(const KParams& kp, size_t lds, int grid, int E, bool qf32, bool vec,
                      hipStream_t s) {
  if (qf32) {
    if (E == 8) return vec ? go_plain<KB, NB, 8, true, true, WPB>(kp, lds, grid, s)
                           : go_plain<KB, NB, 8, true, false, WPB>(kp, lds, grid, s);
    return vec ? go_plain<KB, NB, 4, true, true, WPB>(kp, lds, grid, s)
               : go_plain<KB, NB, 4, true, false, WPB>(kp, lds, grid, s);
  }
  if (E == 8) return vec ? go_plain<KB, NB, 8, false, true, WPB>(kp, lds, grid, s)
                         : go_plain<KB, NB, 8, false, false, WPB>(kp, lds, grid, s);
  return vec ? go_plain<KB, NB, 4, false, true, WPB>(kp, lds, grid, s)
             : go_plain<KB, NB, 4, false, false, WPB>(kp, lds, grid, s);
}

constexpr int kWPB = 4;
constexpr size_t kResidentLds = 96 * 1024;

}  // namespace

hipError_t launch_assign_refined(const AssignArgs& a, hipStream_t s, int n_cu) {
  const DeviceTemplate& t = *a.t;
  const AssignGeom& g = t.geom;
  KParams kp{};
  kp.q = a.q;
  kp.stride = a.stride;
  kp.n_pix = a.n_pix;
  kp.D = a.D;
  kp.frag = t.d_frag_bf16;
  kp.cnorm = t.d_cnorm;
  kp.n_groups = g.d_pad_bf16 / (32 * g.s_bf16);
  kp.labels = a.labels;
  kp.wl_count = a.wl_count;
  kp.wl_pix = a.wl_pix;
  kp.wl_mask = a.wl_mask;
  kp.a0 = a.bound.a0;
  kp.a1 = a.bound.a1;
  kp.a2 = a.bound.a2;
  const bool qf32 = a.dtype == VQNNF_F32;
  const bool vec = rows_aligned(a, qf32 ? 4 : 2);
  const size_t group_bytes = (size_t)g.s_bf16 * 2 * g.kb * 64 * 16;
  const size_t all_bytes = group_bytes * kp.n_groups;
  kp.resident = all_bytes <= kResidentLds;
  const size_t lds = kp.resident ? all_bytes : group_bytes;
  // pixel blocks per wave: KB*NB*4 accumulators stay <= 128 registers
  const int NB = g.kb <= 8 ? 4 : 2;
  const int tile_px = kWPB * NB * 16;
  kp.n_tiles = (a.n_pix + tile_px - 1) / tile_px;
  int grid = (int)std::min<int64_t>(kp.n_tiles, kp.resident ? (int64_t)n_cu * 8 : kp.n_tiles);
  timing_begin(K_ASSIGN_REFINED);
  hipError_t e;
  const int S = g.s_bf16;
  switch (g.kb) {
    case 1: e = go_refined_s<1, 4, kWPB>(kp, lds, grid, S, qf32, vec, s); break;
    case 2: e = go_refined_s<2, 4, kWPB>(kp, lds, grid, S, qf32, vec, s); break;
    case 3: e = go_refined_s<3, 4, kWPB>(kp, lds, grid, S, qf32, vec, s); break;
    case 4: e = go_refined_s<4, 4, kWPB>(kp, lds, grid, S, qf32, vec, s); break;
    case 8: e = go_refined_s<8, 4, kWPB>(kp, lds, grid, S, qf32, vec, s); break;
    case 16: e = go_refined_s<16, 2, kWPB>(kp, lds, grid, S, qf32, vec, s); break;
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
  kp.frag = t.d_frag_f32;
  kp.cnorm = t.d_cnorm;
  kp.n_groups = g.d_pad_f32 / (4 * g.e_f32);
  kp.labels = a.labels;
  const bool qf32 = a.dtype == VQNNF_F32;
  const bool vec = rows_aligned(a, qf32 ? 4 : 2);
  const size_t group_bytes = (size_t)g.e_f32 * g.kb * 64 * 4;
  const size_t all_bytes = group_bytes * kp.n_groups;
  kp.resident = all_bytes <= kResidentLds;
  const size_t lds = kp.resident ? all_bytes : group_bytes;
  const int NB = g.kb <= 8 ? 4 : 2;
  const int tile_px = kWPB * NB * 16;
  kp.n_tiles = (a.n_pix + tile_px - 1) / tile_px;
  int grid = (int)std::min<int64_t>(kp.n_tiles, kp.resident ? (int64_t)n_cu * 8 : kp.n_tiles);
  timing_begin(K_ASSIGN_PLAIN);
  hipError_t e;
  const int E = g.e_f32;
  switch (g.kb) {
    case 1: e = go_plain_s<1, 4, kWPB>(kp, lds, grid, E, qf32, vec, s); break;
    case 2: e = go_plain_s<2, 4, kWPB>(kp, lds, grid, E, qf32, vec, s); break;
    case 3: e = go_plain_s<3, 4, kWPB>(kp, lds, grid, E, qf32, vec, s); break;
    case 4: e = go_plain_s<4, 4, kWPB>(kp, lds, grid, E, qf32, vec, s); break;
    case 8: e = go_plain_s<8, 4, kWPB>(kp, lds, grid, E, qf32, vec, s); break;
    case 16: e = go_plain_s<16, 2, kWPB>(kp, lds, grid, E, qf32, vec, s); break;
    default: e = hipErrorInvalidValue; break;
  }
  timing_end(K_ASSIGN_PLAIN);
  return e;
}

hipError_t launch_rescore(const AssignArgs& a, hipStream_t s, int n_cu) {
  const DeviceTemplate& t = *a.t;
  RParams rp{};
  rp.q = a.q;
  rp.stride = a.stride;
  rp.D = a.D;
  rp.k = t.k;
  rp.mask_words = (t.geom.kpad + 31) / 32;
  rp.qf32 = a.dtype == VQNNF_F32;
  rp.codebook = t.d_codebook;
  rp.wl_count = a.wl_count;
  rp.wl_pix = a.wl_pix;
  rp.wl_mask = a.wl_mask;
  rp.labels = a.labels;
  int grid = n_cu * 4;
  timing_begin(K_RESCORE);
  hipLaunchKernelGGL(rescore_kernel, dim3(grid), dim3(256), 0, s, rp);
  timing_end(K_RESCORE);
  return hipGetLastError();
}

}  // namespace vqnnf
