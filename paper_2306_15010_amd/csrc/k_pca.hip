// Projection of a feature map onto d principal axes (dimensionality
// reduction, Sec. 5.5): out[p][i] = sum_t (q_pt - mean_t) * basis_it, in FP32
// with the subtraction rounded and the products accumulated by FMA
// sequentially in t.
//
// A block owns 64 pixels: the block copies a 64-pixel x 64-element slice of
// the map to LDS with contiguous per-pixel loads (decoding BF16 / FP8 x scale
// / RGB colour patches to FP32), then each of the 4 threads of a pixel
// accumulates a quarter of the d outputs over the slice; the basis and mean
// sit in LDS.  Reading the map from HBM once is the bound.
#include "vqnnf_internal.h"
#include "assign_common.h"

#pragma clang fp contract(off)

namespace vqnnf {

namespace {

constexpr int kPPix = 64;        // pixels per block
constexpr int kPT = 64;          // elements per slice
constexpr int kPMaxOut = 64;     // at most 64 outputs (16 per thread)

struct ProjParams {
  const void* q;
  int64_t stride, n_pix;
  int W, H, D, d;
  const float* scale;          // FP8: [D]
  const float* mean;           // [D]
  const float* basis;          // [d][D]
  float* out;                  // [n_pix][d]
};

template <int QT>
__device__ __forceinline__ float elem(const ProjParams& p, int64_t px, int t) {
  if constexpr (QT == kQF32) {
    return ((const float*)p.q)[px * p.stride + t];
  } else if constexpr (QT == kQBF16) {
    return bf16_bits_to_f32(((const uint16_t*)p.q)[px * p.stride + t]);
  } else if constexpr (QT == kQFP8) {
    const f32x2_t v = __builtin_amdgcn_cvt_pk_f32_fp8((int)((const uint8_t*)p.q)[px * p.stride + t], false);
    return v[0] * p.scale[t];
  } else {
    const int y = (int)(px / p.W), x = (int)(px - (int64_t)y * p.W);
    const int dy = t / 9, dx = (t / 3) % 3, c = t % 3;
    const int yy = min(max(y + dy - 1, 0), p.H - 1), xx = min(max(x + dx - 1, 0), p.W - 1);
    return (float)((const uint8_t*)p.q)[((int64_t)yy * p.W + xx) * p.stride + c];
  }
}

template <int QT>
__global__ __launch_bounds__(256) void pca_project_kernel(ProjParams p) {
  extern __shared__ float sm[];
  float* bs = sm;                                  // [d][D]
  float* ms = bs + p.d * p.D;                      // [D]
  float* qs = ms + p.D;                            // [kPPix][kPT + 1]
  for (int i = threadIdx.x; i < p.d * p.D; i += 256) bs[i] = p.basis[i];
  for (int i = threadIdx.x; i < p.D; i += 256) ms[i] = p.mean[i];
  const int64_t px0 = (int64_t)blockIdx.x * kPPix;
  const int pl = threadIdx.x >> 2, part = threadIdx.x & 3;
  const int per = (p.d + 3) / 4;                   // outputs of this thread: part*per ..
  const int o0 = part * per, o1 = min(p.d, o0 + per);
  float acc[kPMaxOut / 4];
#pragma unroll
  for (int i = 0; i < kPMaxOut / 4; ++i) acc[i] = 0.f;
  for (int t0 = 0; t0 < p.D; t0 += kPT) {
    const int tn = min(kPT, p.D - t0);
    __syncthreads();
    for (int e = threadIdx.x; e < kPPix * kPT; e += 256) {
      const int r = e / kPT, t = e % kPT;
      const int64_t px = min(px0 + r, p.n_pix - 1);
      qs[r * (kPT + 1) + t] = t < tn ? elem<QT>(p, px, t0 + t) - ms[t0 + t] : 0.f;
    }
    __syncthreads();
    const float* qr = qs + pl * (kPT + 1);
    for (int t = 0; t < tn; ++t) {
      const float qv = qr[t];
#pragma unroll
      for (int i = 0; i < kPMaxOut / 4; ++i)
        if (o0 + i < o1) acc[i] = __builtin_fmaf(qv, bs[(o0 + i) * p.D + t0 + t], acc[i]);
    }
  }
  const int64_t px = px0 + pl;
  if (px < p.n_pix)
    for (int i = 0; i < kPMaxOut / 4; ++i)
      if (o0 + i < o1) p.out[px * p.d + o0 + i] = acc[i];
}

}  // namespace

size_t pca_project_lds(int D, int d) { return ((size_t)d * D + D + (size_t)kPPix * (kPT + 1)) * sizeof(float); }

hipError_t launch_pca_project(const void* q, int dtype, int64_t stride, int H, int W, int D, const float* scale,
                              const float* mean, const float* basis, int d, float* out, hipStream_t s) {
  ProjParams p{};
  p.q = q;
  p.stride = stride;
  p.n_pix = (int64_t)H * W;
  p.W = W;
  p.H = H;
  p.D = D;
  p.d = d;
  p.scale = scale;
  p.mean = mean;
  p.basis = basis;
  p.out = out;
  const size_t lds = pca_project_lds(D, d);
  const dim3 grid((unsigned)((p.n_pix + kPPix - 1) / kPPix));
  auto go = [&](auto kern) -> hipError_t {
    if (lds > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, p);
    return hipGetLastError();
  };
  timing_begin(K_PCA_PROJECT);
  hipError_t e;
  if (dtype == VQNNF_F32) e = go(pca_project_kernel<kQF32>);
  else if (dtype == VQNNF_BF16) e = go(pca_project_kernel<kQBF16>);
  else if (dtype == VQNNF_FP8_E4M3) e = go(pca_project_kernel<kQFP8>);
  else e = go(pca_project_kernel<kQRGB8>);
  timing_end(K_PCA_PROJECT);
  return e;
}

}  // namespace vqnnf
