// Score of a bank with weighted coarse filters (Sec. 3.2.1 eq. 1 with
// Alg. 2's dilation taps, Sec. 3.2.2, Sec. 3.3 eq. 2) plus localisation
// (Sec. 4), from the one-hot integral image P (exclusive, channel-last).
//
// For a region group with gx x gy bins whose edges sit at offsets X_a, Y_b
// from the window's top-left (x, y), the taps P[y+Y_b][x+X_a] give every bin
// count exactly in integers,
//   n_j(a, b) = (P[Y_b+1][X_a+1] - P[Y_b+1][X_a]) - (P[Y_b][X_a+1] - P[Y_b][X_a]),
// which is Alg. 2's dilation filter applied per bin before the weights; a
// filter's response is then the FP32 FMA chain sum_{b,a} coef(a,b) * n_j(a,b)
// over its non-zero bins in row-major order (the host evaluates R(tau) with
// the same chain, so a window identical to the template scores exactly 0).
// Eq. 2 per window: -sum_f w_f * sum_j |R_f,j(tau) - R_f,j(q)|.
//
// Taps come either from a 32-bit P (vqnnf_filter's output) or from P stored
// mod 2^16 with an even channel count (the matching path): a bin count is
// below 2^16, so the wrapping 16-bit differences are exact, and one 32-bit
// load brings a channel pair.  Both variants give the same channel pairs to
// the same lanes and sum in the same order, so their heatmaps are identical.
//
// A window is owned by L = min(64, next pow2 >= channel pairs) lanes (64/L
// windows per wave-iteration); lane c holds pairs c, c+L, ...  A wave walks
// `iters` consecutive window-iterations; the flat stream of (window, group)
// steps is software-pipelined: the next step's taps are requested before the
// current step's arithmetic.  Every tap is loaded for a G x G grid (edges past
// a group's own grid repeat its last edge and have zero coefficients), so the
// number of loads per step is fixed and the waits are exact.
#include "vqnnf_internal.h"
#include "dev_common.h"
#include "assign_common.h"

namespace vqnnf {

namespace {

typedef unsigned short u16x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ unsigned long long bank_key(float score, uint32_t idx) {
  uint32_t b = __float_as_uint(score);
  uint32_t o = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  return ((unsigned long long)o << 32) | (unsigned long long)(0xFFFFFFFFu - idx);
}

__device__ __forceinline__ void bank_block_max(unsigned long long key, unsigned long long* best) {
  __shared__ unsigned long long wmax[4];
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    unsigned long long o = __shfl_xor(key, m);
    key = o > key ? o : key;
  }
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = key;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = wmax[0];
    for (int i = 1; i < 4; ++i) m = wmax[i] > m ? wmax[i] : m;
    if (m > __hip_atomic_load(best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(best, m);
  }
}

struct BankParams {
  const void* P;             // int32 [(H+1)][(W+1)][k], or u16 [(H+1)][(W+1)][2*npairs]
  int k, ow, oh, npairs;
  int64_t row;               // 32-bit words per P row
  int64_t pix;               // 32-bit words per P entry (k, or npairs)
  int ng, kpad, lg, iters, nf;
  const BankGroup* groups;
  const float* coef;         // [nf][16]
  const float* resp;         // [nf][kpad]
  const float* fw;           // [nf]
  float* heatmap;
  unsigned long long* best;
};

// T16: taps are u16 pairs; CPL: channel pairs per lane; G: taps per side - 1.
// The read-only tables are separate restrict arguments so that their
// wave-uniform reads become scalar loads.
template <bool T16, int CPL, int G>
__global__ __launch_bounds__(256) void score_bank_kernel(BankParams p, const BankGroup* __restrict__ groups,
                                                         const float* __restrict__ coef,
                                                         const float* __restrict__ fw) {
  constexpr int NV = T16 ? 1 : 2;              // 32-bit words per pair
  const int lane = threadIdx.x & 63;
  const int L = 1 << p.lg;
  const int cl = lane & (L - 1);
  const int sub = lane >> p.lg;
  const int64_t nwin = (int64_t)p.ow * p.oh;
  const int64_t wave_id = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int ng = p.ng;
  const int nsteps = p.iters * ng;
  int po[CPL][NV];                             // word offset of each channel in a P entry
  int pq[CPL];                                 // pair index (clamped)
  bool cv0[CPL], cv1[CPL];                     // channel 2q / 2q+1 exists
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    const int q = cl + c * L;
    const bool pv = q < p.npairs;
    const int qc = pv ? q : p.npairs - 1;
    pq[c] = qc;
    cv0[c] = pv && 2 * q < p.k;
    cv1[c] = pv && 2 * q + 1 < p.k;
    if (T16) {
      po[c][0] = qc;
    } else {
      po[c][0] = min(2 * qc, p.k - 1);
      if (NV > 1) po[c][NV - 1] = min(2 * qc + 1, p.k - 1);
    }
  }
  const uint32_t* P = (const uint32_t*)p.P;
  // R(tau), bin coefficients and filter weights in LDS: their reads then do
  // not wait behind the tap loads in flight
  extern __shared__ float rs[];  // [nf][kpad] R(tau)
  for (int i = threadIdx.x; i < p.nf * p.kpad; i += 256) rs[i] = p.resp[i];
  __syncthreads();

  typedef uint32_t Taps[G + 1][G + 1][CPL][NV];
  auto win_of = [&](int it) -> int64_t {
    return (((wave_id * p.iters + it) << (6 - p.lg))) + sub;
  };
  // Taps through a buffer resource based at the P row of the step's first
  // window: per lane one 32-bit offset per step, per tap a scalar offset
  // (every offset inside a band of h + 2 rows of P stays below 2^32).
  auto load = [&](int it, int gi, Taps& t) {
    const int64_t w = win_of(it);
    const int wc = (int)(w < nwin ? w : nwin - 1);  // clamped: every tap stays inside P
    const int64_t w0 = win_of(it) - sub;
    const int w0c = __builtin_amdgcn_readfirstlane((int)(w0 < nwin ? w0 : nwin - 1));
    const int y0 = w0c / p.ow;
    const int y = wc / p.ow, x = wc - y * p.ow;
    const __amdgpu_buffer_rsrc_t rsrc = raw_rsrc(P + (int64_t)y0 * p.row);
    const uint32_t vb = ((uint32_t)(y - y0) * (uint32_t)p.row + (uint32_t)x * (uint32_t)p.pix) * 4u;
    const BankGroup& g = groups[gi];
    const uint32_t rowb = (uint32_t)p.row * 4u, pixb = (uint32_t)p.pix * 4u;
#pragma unroll
    for (int tb = 0; tb <= G; ++tb) {
      const uint32_t ro = (uint32_t)g.ye[tb] * rowb;
#pragma unroll
      for (int ta = 0; ta <= G; ++ta) {
        const uint32_t so = ro + (uint32_t)g.xe[ta] * pixb;
#pragma unroll
        for (int c = 0; c < CPL; ++c)
#pragma unroll
          for (int v = 0; v < NV; ++v)
            t[tb][ta][c][v] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, vb + 4u * (uint32_t)po[c][v], so, 0);
      }
    }
  };
  float acc = 0.f;
  unsigned long long key = 0ull;
  auto compute = [&](int it, int gi, const Taps& t) {
    const BankGroup& g = groups[gi];
    float cnt[G][G][CPL][2];
#pragma unroll
    for (int b = 0; b < G; ++b)
#pragma unroll
      for (int a = 0; a < G; ++a)
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
          if (T16) {
            const u16x2_t d = (__builtin_bit_cast(u16x2_t, t[b + 1][a + 1][c][0]) -
                               __builtin_bit_cast(u16x2_t, t[b + 1][a][c][0])) -
                              (__builtin_bit_cast(u16x2_t, t[b][a + 1][c][0]) -
                               __builtin_bit_cast(u16x2_t, t[b][a][c][0]));
            cnt[b][a][c][0] = (float)d.x;
            cnt[b][a][c][1] = (float)d.y;
          } else {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int v = NV > 1 ? h : 0;
              const int d = ((int)t[b + 1][a + 1][c][v] - (int)t[b + 1][a][c][v]) -
                            ((int)t[b][a + 1][c][v] - (int)t[b][a][c][v]);
              cnt[b][a][c][h] = (float)d;
            }
          }
        }
    for (int f = g.f0; f < g.f1; ++f) {
      const float* cf = (const float*)__builtin_assume_aligned(coef + f * 16, 64);
      float r[CPL][2];
#pragma unroll
      for (int c = 0; c < CPL; ++c) r[c][0] = r[c][1] = 0.f;
#pragma unroll
      for (int b = 0; b < G; ++b)
#pragma unroll
        for (int a = 0; a < G; ++a) {
          // a zero coefficient leaves the chain unchanged (fma(0, n, r) = r for
          // a finite count n), so every bin takes part: no branch per bin
          const float cv = cf[b * 4 + a];
#pragma unroll
          for (int c = 0; c < CPL; ++c) {
            r[c][0] = __builtin_fmaf(cv, cnt[b][a][c][0], r[c][0]);
            r[c][1] = __builtin_fmaf(cv, cnt[b][a][c][1], r[c][1]);
          }
        }
      const float* rt = rs + f * p.kpad;
      float l1 = 0.f;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const float2 tv = *(const float2*)(rt + 2 * pq[c]);
        const float d0 = __builtin_fabsf(tv.x - r[c][0]);
        const float d1 = __builtin_fabsf(tv.y - r[c][1]);
        l1 += cv0[c] ? d0 : 0.f;
        l1 += cv1[c] ? d1 : 0.f;
      }
      acc = __builtin_fmaf(fw[f], l1, acc);
    }
    if (gi == ng - 1) {
      float v = acc;
      for (int m = 1; m < L; m <<= 1) v += __shfl_xor(v, m);
      const int64_t w = win_of(it);
      if (w < nwin && cl == 0) {
        const float score = -v;
        p.heatmap[w] = score;
        const unsigned long long k2 = bank_key(score, (uint32_t)w);
        key = k2 > key ? k2 : key;
      }
      acc = 0.f;
    }
  };
  // loads per step; a wait for "all but the next step's loads" needs that
  // count to fit the counter (else wait for everything)
  constexpr int LPS = (G + 1) * (G + 1) * CPL * NV;
  constexpr int WN = LPS <= 63 ? LPS : 0;
  Taps ta, tb;
  // (window, group) cursors of steps s and s + 1, advanced without divisions
  auto advance = [&](int& it, int& gi) {
    if (++gi == ng) {
      gi = 0;
      ++it;
    }
  };
  if (win_of(0) - sub < nwin) {                // uniform per wave
    int ci = 0, cg = 0, ni = 0, ngi = 0;
    advance(ni, ngi);
    load(0, 0, ta);
    for (int s = 0; s < nsteps; s += 2) {
      const bool h1 = s + 1 < nsteps;
      load(h1 ? ni : ci, h1 ? ngi : cg, tb);   // always issued: the count stays fixed
      __builtin_amdgcn_sched_barrier(0);
      wait_vm<WN>();
      __builtin_amdgcn_sched_barrier(0);
      compute(ci, cg, ta);
      if (h1) {
        int i2 = ni, g2 = ngi;
        advance(i2, g2);
        const bool h2 = s + 2 < nsteps;
        load(h2 ? i2 : ni, h2 ? g2 : ngi, ta);
        __builtin_amdgcn_sched_barrier(0);
        wait_vm<WN>();
        __builtin_amdgcn_sched_barrier(0);
        compute(ni, ngi, tb);
        ci = i2;
        cg = g2;
        ni = i2;
        ngi = g2;
        advance(ni, ngi);
      }
    }
    wait_vm<0>();
  }
  bank_block_max(key, p.best);
}

template <bool T16, int CPL, int G>
hipError_t go_bank_g(const BankParams& bp, dim3 grid, size_t lds, hipStream_t s) {
  auto kern = score_bank_kernel<T16, CPL, G>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, bp, bp.groups, bp.coef, bp.fw);
  return hipGetLastError();
}

template <bool T16, int CPL>
hipError_t go_bank(const BankParams& bp, int G, dim3 grid, size_t lds, hipStream_t s) {
  if (G <= 1) return go_bank_g<T16, CPL, 1>(bp, grid, lds, s);
  if (G == 2) return go_bank_g<T16, CPL, 2>(bp, grid, lds, s);
  if (G == 3) return go_bank_g<T16, CPL, 3>(bp, grid, lds, s);
  return go_bank_g<T16, CPL, 4>(bp, grid, lds, s);
}

}  // namespace

hipError_t launch_score_bank(const ScoreArgs& a, hipStream_t s) {
  const DeviceTemplate& t = *a.t;
  const bool t16 = a.P16 != nullptr;
  BankParams bp{};
  bp.P = t16 ? (const void*)a.P16 : (const void*)a.P;
  bp.k = t.k;
  bp.ow = a.W - t.w + 1;
  bp.oh = a.H - t.h + 1;
  bp.npairs = (t.k + 1) / 2;
  bp.pix = t16 ? bp.npairs : t.k;
  bp.row = (int64_t)(a.W + 1) * bp.pix;
  bp.ng = (int)t.groups.size();
  bp.kpad = t.geom.kpad;
  bp.nf = t.n_filters;
  const size_t lds = (size_t)t.n_filters * t.geom.kpad * sizeof(float);
  int lg = 0;
  while ((1 << lg) < bp.npairs && lg < 6) ++lg;
  bp.lg = lg;
  const int cpl = (bp.npairs + (1 << lg) - 1) >> lg;   // 1 or 2 (k <= 256)
  bp.groups = t.d_groups;
  bp.coef = t.d_coef;
  bp.resp = t.d_resp;
  bp.fw = t.d_weights;
  bp.heatmap = a.heatmap;
  bp.best = a.best;
  const int64_t nwin = (int64_t)bp.ow * bp.oh;
  const int64_t wpi = 64 >> lg;                        // windows per wave-iteration
  // enough waves for every CU, at most 16 window-iterations each
  const int64_t target_waves = 256ll * 32;
  int64_t iters = (nwin + wpi * target_waves - 1) / (wpi * target_waves);
  iters = std::max<int64_t>(1, std::min<int64_t>(16, iters));
  bp.iters = (int)iters;
  const int64_t waves = (nwin + wpi * iters - 1) / (wpi * iters);
  const dim3 grid((unsigned)((waves + 3) / 4));
  timing_begin(K_SCORE_BANK);
  hipError_t e;
  if (t16) {
    e = cpl == 1 ? go_bank<true, 1>(bp, t.bank_g, grid, lds, s) : go_bank<true, 2>(bp, t.bank_g, grid, lds, s);
  } else {
    e = cpl == 1 ? go_bank<false, 1>(bp, t.bank_g, grid, lds, s) : go_bank<false, 2>(bp, t.bank_g, grid, lds, s);
  }
  timing_end(K_SCORE_BANK);
  return e;
}

}  // namespace vqnnf
