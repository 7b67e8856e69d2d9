// Nearest-codeword assignment (Alg. 1, Sec. 3.1) for low-dimensional features
// (D <= 32: the PCA-reduced features of Sec. 5.5) and for colour features
// built on the fly from an RGB image (Sec. 5.2 "Feature Extraction": the 3x3
// neighbourhood of RGB values, D = 27, edges replicated).
//
// Two pixels per thread: their features in registers, the codebook read through
// scalar loads (the same value for every lane: an SGPR operand of the FMA), the
// direct distances d~_j = sum_t (q_t - c_jt)^2 in FP32 (subtract, then FMA).
// Their error is relative: |d~_j - d_j| <= e32 * d_j with
// e32 = (1 + u)^2 (1 + gamma_D) - 1, u = 2^-24, and the FP64 distances of the
// exact rule satisfy |o_j - d_j| <= e64 * d_j likewise.  With
// tau >= (e32 + e64) (1 + 2^-10), a pixel whose two smallest d~ satisfy
// d~2 - d~1 > tau (d~1 + d~2) has o_j > o_j1 for every other codeword, so j1 is
// the exact label; otherwise the pixel goes to the FP64 re-score with the
// candidates j for which d~_j - d~1 <= tau (d~1 + d~_j) (every other codeword
// has an FP64 distance above j1's).  A small absolute floor covers values
// below the normal range.
#include "vqnnf_internal.h"
#include "assign_common.h"

#pragma clang fp contract(off)

namespace vqnnf {

namespace {

constexpr int kLowMaxD = 32;

struct LowParams {
  const void* q;
  int64_t stride;          // elements (bytes for RGB) between pixels
  int64_t n_pix;
  int W, H, D, k, mask_words, refined;
  uint8_t* labels;
  uint32_t* wl_count;
  uint32_t* wl_pix;
  uint32_t* wl_mask;
  float tau, floor;
};

template <int QT>
__device__ __forceinline__ void load_features(const LowParams& p, int64_t px, float (&qv)[kLowMaxD]) {
  if constexpr (QT == kQRGB8) {
    const uint8_t* img = (const uint8_t*)p.q;
    const int y = (int)(px / p.W), x = (int)(px - (int64_t)y * p.W);
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const int yy = min(max(y + dy - 1, 0), p.H - 1);
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int xx = min(max(x + dx - 1, 0), p.W - 1);
        const uint8_t* px8 = img + ((int64_t)yy * p.W + xx) * p.stride;
#pragma unroll
        for (int c = 0; c < 3; ++c) qv[(3 * dy + dx) * 3 + c] = (float)px8[c];
      }
    }
#pragma unroll
    for (int t = 27; t < kLowMaxD; ++t) qv[t] = 0.f;
  } else {
#pragma unroll
    for (int t = 0; t < kLowMaxD; ++t) {
      float v = 0.f;
      if (t < p.D) {
        if constexpr (QT == kQF32) v = ((const float*)p.q)[px * p.stride + t];
        else v = bf16_bits_to_f32(((const uint16_t*)p.q)[px * p.stride + t]);
      }
      qv[t] = v;
    }
  }
}

// DT > 0: the feature size as a compile-time constant (no per-element test).
template <int DT>
__device__ __forceinline__ float dist(const float (&qv)[kLowMaxD], const float* __restrict__ c, int D) {
  float d = 0.f;
#pragma unroll
  for (int t = 0; t < (DT > 0 ? DT : kLowMaxD); ++t) {
    if (DT > 0 || t < D) {
      const float diff = qv[t] - c[t];
      d = __builtin_fmaf(diff, diff, d);
    }
  }
  return d;
}

// Two pixels per thread (px and px + 256 of a block's 512): every codeword
// value read through a scalar load serves both.
template <int QT, int DT>
__global__ __launch_bounds__(256) void assign_lowd_kernel(LowParams p, const float* __restrict__ cb) {
  constexpr int PPT = 2;
  float qv[PPT][kLowMaxD];
  int64_t px[PPT];
  bool valid[PPT];
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    px[u] = (int64_t)blockIdx.x * (256 * PPT) + 256 * u + threadIdx.x;
    valid[u] = px[u] < p.n_pix;
    load_features<QT>(p, valid[u] ? px[u] : p.n_pix - 1, qv[u]);
  }
  const int D = DT > 0 ? DT : p.D;
  float d1[PPT], d2[PPT];
  int j1[PPT];
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    d1[u] = __builtin_inff();
    d2[u] = __builtin_inff();
    j1[u] = 0;
  }
  for (int j = 0; j < p.k; ++j) {
    const float* c = cb + j * D;
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      // first index on ties: equal values never displace the best
      const float d = dist<DT>(qv[u], c, D);
      const bool lt1 = d < d1[u], lt2 = d < d2[u];
      d2[u] = lt1 ? d1[u] : (lt2 ? d : d2[u]);
      j1[u] = lt1 ? j : j1[u];
      d1[u] = lt1 ? d : d1[u];
    }
  }
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    if (valid[u]) p.labels[px[u]] = (uint8_t)j1[u];
    if (!p.refined) continue;
    const bool flag = valid[u] && p.k > 1 && (d2[u] - d1[u] <= p.tau * (d1[u] + d2[u]) + p.floor);
    const uint64_t bal = __ballot(flag);
    if (bal == 0) continue;
    uint32_t base = 0;
    const int leader = __builtin_amdgcn_readfirstlane(__ffsll((long long)bal) - 1);
    if (lane == leader) base = atomicAdd(p.wl_count, (uint32_t)__popcll(bal));
    base = __shfl(base, leader);
    if (!flag) continue;
    const uint32_t pos = base + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
    p.wl_pix[pos] = (uint32_t)px[u];
    for (int w = 0; w < p.mask_words; ++w) {
      uint32_t bits = 0u;
      for (int b = 0; b < 32; ++b) {
        const int j = 32 * w + b;
        if (j >= p.k) break;
        const float d = dist<DT>(qv[u], cb + j * D, D);
        if (d - d1[u] <= p.tau * (d1[u] + d) + p.floor) bits |= 1u << b;
      }
      p.wl_mask[(int64_t)pos * p.mask_words + w] = bits;
    }
  }
}

template <int QT>
void go_lowd(const LowParams& p, const float* cb, int D, hipStream_t s) {
  const dim3 grid((unsigned)((p.n_pix + 511) / 512));
  switch (D) {
    case 9: hipLaunchKernelGGL((assign_lowd_kernel<QT, 9>), grid, dim3(256), 0, s, p, cb); break;
    case 18: hipLaunchKernelGGL((assign_lowd_kernel<QT, 18>), grid, dim3(256), 0, s, p, cb); break;
    case 27: hipLaunchKernelGGL((assign_lowd_kernel<QT, 27>), grid, dim3(256), 0, s, p, cb); break;
    default: hipLaunchKernelGGL((assign_lowd_kernel<QT, 0>), grid, dim3(256), 0, s, p, cb); break;
  }
}

}  // namespace

bool lowd_supported(int dtype, int D) {
  return dtype == VQNNF_RGB8 || ((dtype == VQNNF_F32 || dtype == VQNNF_BF16) && D <= kLowMaxD);
}

hipError_t launch_assign_lowd(const AssignArgs& a, bool refined, hipStream_t s) {
  const DeviceTemplate& t = *a.t;
  LowParams p{};
  p.q = a.q;
  p.stride = a.stride;
  p.n_pix = a.n_pix;
  p.W = a.img_w;
  p.H = a.img_h;
  p.D = a.D;
  p.k = t.k;
  p.mask_words = (t.geom.kpad + 31) / 32;
  p.refined = refined ? 1 : 0;
  p.labels = a.labels;
  p.wl_count = a.wl_count;
  p.wl_pix = a.wl_pix;
  p.wl_mask = a.wl_mask;
  // e32 and e64 as above (gamma_n = n u / (1 - n u)), tau with a 2^-10 margin
  const double u32 = 0x1.0p-24, u64 = 0x1.0p-53, D = a.D;
  const double g32 = D * u32 / (1.0 - D * u32), g64 = (D + 2) * u64 / (1.0 - (D + 2) * u64);
  const double e32 = (1.0 + u32) * (1.0 + u32) * (1.0 + g32) - 1.0;
  const double e64 = (1.0 + u64) * (1.0 + u64) * (1.0 + g64) - 1.0;
  p.tau = (float)((e32 + e64) * (1.0 + 0x1.0p-10) * (1.0 + 0x1.0p-20));
  p.floor = (float)(4.0 * (D + 2) * 0x1.0p-126);
  timing_begin(K_ASSIGN_LOWD);
  const float* cb = t.d_codebook;
  if (a.dtype == VQNNF_RGB8) go_lowd<kQRGB8>(p, cb, 27, s);
  else if (a.dtype == VQNNF_F32) go_lowd<kQF32>(p, cb, a.D, s);
  else go_lowd<kQBF16>(p, cb, a.D, s);
  timing_end(K_ASSIGN_LOWD);
  return hipGetLastError();
}

}  // namespace vqnnf
