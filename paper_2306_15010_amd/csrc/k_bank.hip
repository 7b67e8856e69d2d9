// Score of a bank with weighted coarse filters (Sec. 3.2.1 eq. 1 with
// Alg. 2's dilation taps, Sec. 3.2.2, Sec. 3.3 eq. 2) plus localisation
// (Sec. 4), from the one-hot integral image P (exclusive, channel-last).
//
// For a region group with gx x gy bins whose edges sit at offsets X_a, Y_b
// from the window's top-left (x, y), the (gx+1)(gy+1) taps P[y+Y_b][x+X_a]
// give every bin count exactly in integers,
//   n_j(a, b) = (P[Y_b+1][X_a+1] - P[Y_b+1][X_a]) - (P[Y_b][X_a+1] - P[Y_b][X_a]),
// which is Alg. 2's dilation filter applied per bin before the weights; a
// filter's response is then the FP32 FMA chain sum_{b,a} coef(a,b) * n_j(a,b)
// over its non-zero bins in row-major order (the host evaluates R(tau) with
// the same chain, so a window identical to the template scores exactly 0).
// Eq. 2 per window: -sum_f w_f * sum_j |R_f,j(tau) - R_f,j(q)|.
//
// A window is owned by L = min(64, next pow2 >= k) lanes of a wave (64/L
// windows per wave); lane c holds channels c, c+L, ..., so every tap load of
// a wave reads L consecutive int32 of one or several adjacent P entries.
#include "vqnnf_internal.h"
#include "dev_common.h"

namespace vqnnf {

namespace {

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
  const int32_t* P;
  int k, ow, oh;
  int64_t row;               // (W + 1) * k
  int ng, kpad, lpw_log2;
  const BankGroup* groups;
  const float* coef;         // [nf][16]
  const float* resp;         // [nf][kpad]
  const float* fw;           // [nf]
  float* heatmap;
  unsigned long long* best;
};

template <int CPL>
__global__ __launch_bounds__(256) void score_bank_kernel(BankParams p) {
  const int lane = threadIdx.x & 63;
  const int L = 1 << p.lpw_log2;
  const int cl = lane & (L - 1);
  const int64_t nwin = (int64_t)p.ow * p.oh;
  const int64_t win = (((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) << (6 - p.lpw_log2)) + (lane >> p.lpw_log2);
  const bool valid = win < nwin;
  const int64_t wc = valid ? win : nwin - 1;      // clamped: every tap stays inside P
  const int x = (int)(wc % p.ow), y = (int)(wc / p.ow);
  int jj[CPL];
  bool jv[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    const int j = cl + c * L;
    jv[c] = j < p.k;
    jj[c] = jv[c] ? j : p.k - 1;
  }
  const int32_t* base = p.P + (int64_t)y * p.row + (int64_t)x * p.k;
  float acc = 0.f;
  for (int gi = 0; gi < p.ng; ++gi) {
    const BankGroup& G = p.groups[gi];
    const int gx = G.gx, gy = G.gy;
    float cnt[kBankMaxG][kBankMaxG][CPL];
    int dprev[kBankMaxG][CPL];
#pragma unroll
    for (int tb = 0; tb <= kBankMaxG; ++tb) {
      if (tb > gy) break;
      const int32_t* rp = base + (int64_t)G.ye[tb] * p.row;
      int t[kBankMaxG + 1][CPL];
#pragma unroll
      for (int ta = 0; ta <= kBankMaxG; ++ta) {
        if (ta > gx) break;
        const int32_t* cp = rp + (int64_t)G.xe[ta] * p.k;
#pragma unroll
        for (int c = 0; c < CPL; ++c) t[ta][c] = cp[jj[c]];
      }
#pragma unroll
      for (int a = 0; a < kBankMaxG; ++a) {
        if (a >= gx) break;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
          const int d = t[a + 1][c] - t[a][c];
          if (tb > 0) cnt[tb - 1][a][c] = (float)(d - dprev[a][c]);
          dprev[a][c] = d;
        }
      }
    }
    for (int f = G.f0; f < G.f1; ++f) {
      const float* cf = p.coef + f * 16;
      float r[CPL];
#pragma unroll
      for (int c = 0; c < CPL; ++c) r[c] = 0.f;
#pragma unroll
      for (int b = 0; b < kBankMaxG; ++b) {
        if (b >= gy) break;
#pragma unroll
        for (int a = 0; a < kBankMaxG; ++a) {
          if (a >= gx) break;
          const float cv = cf[b * 4 + a];
          if (cv != 0.f) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) r[c] = __builtin_fmaf(cv, cnt[b][a][c], r[c]);
          }
        }
      }
      const float* rt = p.resp + (int64_t)f * p.kpad;
      float l1 = 0.f;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const float d = __builtin_fabsf(rt[jj[c]] - r[c]);
        l1 += jv[c] ? d : 0.f;
      }
      acc = __builtin_fmaf(p.fw[f], l1, acc);
    }
  }
  for (int m = 1; m < L; m <<= 1) acc += __shfl_xor(acc, m);
  unsigned long long key = 0ull;
  if (valid && cl == 0) {
    const float score = -acc;
    p.heatmap[win] = score;
    key = bank_key(score, (uint32_t)win);
  }
  bank_block_max(key, p.best);
}

}  // namespace

hipError_t launch_score_bank(const ScoreArgs& a, hipStream_t s) {
  const DeviceTemplate& t = *a.t;
  BankParams bp{};
  bp.P = a.P;
  bp.k = t.k;
  bp.ow = a.W - t.w + 1;
  bp.oh = a.H - t.h + 1;
  bp.row = (int64_t)(a.W + 1) * t.k;
  bp.ng = (int)t.groups.size();
  bp.kpad = t.geom.kpad;
  int L = 1;
  while (L < t.k && L < 64) L <<= 1;
  int lg = 0;
  while ((1 << lg) < L) ++lg;
  bp.lpw_log2 = lg;
  const int cpl = (t.k + L - 1) / L;
  bp.groups = t.d_groups;
  bp.coef = t.d_coef;
  bp.resp = t.d_resp;
  bp.fw = t.d_weights;
  bp.heatmap = a.heatmap;
  bp.best = a.best;
  const int64_t nwin = (int64_t)bp.ow * bp.oh;
  const int64_t per_block = 4ll * (64 / L);
  const dim3 grid((unsigned)((nwin + per_block - 1) / per_block)), blk(256);
  timing_begin(K_SCORE_BANK);
  if (cpl == 1) hipLaunchKernelGGL(score_bank_kernel<1>, grid, blk, 0, s, bp);
  else if (cpl == 2) hipLaunchKernelGGL(score_bank_kernel<2>, grid, blk, 0, s, bp);
  else hipLaunchKernelGGL(score_bank_kernel<4>, grid, blk, 0, s, bp);
  timing_end(K_SCORE_BANK);
  return hipGetLastError();
}

}  // namespace vqnnf
