// Projection of a feature map onto d principal axes (dimensionality
// reduction, Sec. 5.5): out[p][i] = sum_t (q_pt - mean_t) * basis_it, in FP32
// with the subtraction rounded and the products accumulated by FMA
// sequentially in t (FP8 elements are code x scale rounded to FP32 first).
//
// One thread per pixel with its d outputs in registers.  The pixel's row is
// read in chunks of 8 elements (16-byte loads when rows are aligned, the next
// chunk in flight while one is used); the basis (stored t-major, d values per
// element) and the mean are the same for every lane and come through scalar
// loads as FMA operands.  Reading the map once from HBM and the d FMAs per
// element bound it.  BF16 maps with aligned rows of whole 32-element groups
// take the matrix-core kernel below instead.
#include "vqnnf_internal.h"
#include "assign_common.h"

#pragma clang fp contract(off)

namespace vqnnf {

namespace {

struct ProjParams {
  const void* q;
  int64_t stride, n_pix;
  int W, H, D, d;
  float* out;                  // [n_pix][d]
};

template <int DO>
__device__ __forceinline__ void accumulate(float v, const float* __restrict__ b, int d, float (&acc)[DO]) {
#pragma unroll
  for (int i = 0; i < DO; ++i)
    if (i < d) acc[i] = __builtin_fmaf(v, b[i], acc[i]);
}

// 8 elements of a row as FP32 (QT: F32 / BF16 / FP8 codes times scale).
template <int QT, bool VEC>
__device__ __forceinline__ void load8(const ProjParams& p, int64_t px, int t0, const float* __restrict__ scale,
                                      float (&v)[8]) {
  if constexpr (VEC) {
    if constexpr (QT == kQF32) {
      const uint4* r = (const uint4*)((const float*)p.q + px * p.stride + t0);
      const uint4 a = r[0], b = r[1];
      const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = __uint_as_float(w[e]);
    } else if constexpr (QT == kQBF16) {
      const uint4 a = *(const uint4*)((const uint16_t*)p.q + px * p.stride + t0);
      const uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        v[2 * e] = __uint_as_float(w[e] << 16);
        v[2 * e + 1] = __uint_as_float(w[e] & 0xFFFF0000u);
      }
    } else {
      const uint2 a = *(const uint2*)((const uint8_t*)p.q + px * p.stride + t0);
      float x[8];
      fp8x8_to_f32(a.x, a.y, x);
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = x[e] * scale[t0 + e];
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int t = min(t0 + e, p.D - 1);
      if constexpr (QT == kQF32) {
        v[e] = ((const float*)p.q)[px * p.stride + t];
      } else if constexpr (QT == kQBF16) {
        v[e] = bf16_bits_to_f32(((const uint16_t*)p.q)[px * p.stride + t]);
      } else {
        const f32x2_t c = __builtin_amdgcn_cvt_pk_f32_fp8((int)((const uint8_t*)p.q)[px * p.stride + t], false);
        v[e] = c[0] * scale[t];
      }
    }
  }
}

template <int QT, bool VEC, int DO>
__global__ __launch_bounds__(256) void pca_project_kernel(ProjParams p, const float* __restrict__ bt,
                                                          const float* __restrict__ mean,
                                                          const float* __restrict__ scale) {
  const int64_t px = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t pc = px < p.n_pix ? px : p.n_pix - 1;
  const int d = p.d;
  float acc[DO];
#pragma unroll
  for (int i = 0; i < DO; ++i) acc[i] = 0.f;
  if constexpr (QT == kQRGB8) {
    const uint8_t* img = (const uint8_t*)p.q;
    const int y = (int)(pc / p.W), x = (int)(pc - (int64_t)y * p.W);
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const int yy = min(max(y + dy - 1, 0), p.H - 1);
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int xx = min(max(x + dx - 1, 0), p.W - 1);
        const uint8_t* px8 = img + ((int64_t)yy * p.W + xx) * p.stride;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int t = (3 * dy + dx) * 3 + c;
          accumulate<DO>((float)px8[c] - mean[t], bt + t * d, d, acc);
        }
      }
    }
  } else {
    const int nc = p.D / 8;                  // whole chunks of 8 elements
    float va[8], vb[8];
    if (nc > 0) load8<QT, VEC>(p, pc, 0, scale, va);
    for (int c = 0; c < nc; c += 2) {
      if (c + 1 < nc) load8<QT, VEC>(p, pc, 8 * (c + 1), scale, vb);
#pragma unroll
      for (int e = 0; e < 8; ++e) accumulate<DO>(va[e] - mean[8 * c + e], bt + (8 * c + e) * d, d, acc);
      if (c + 1 < nc) {
        if (c + 2 < nc) load8<QT, VEC>(p, pc, 8 * (c + 2), scale, va);
#pragma unroll
        for (int e = 0; e < 8; ++e)
          accumulate<DO>(vb[e] - mean[8 * (c + 1) + e], bt + (8 * (c + 1) + e) * d, d, acc);
      }
    }
    for (int t = 8 * nc; t < p.D; ++t) {     // tail
      float v;
      if constexpr (QT == kQF32) {
        v = ((const float*)p.q)[pc * p.stride + t];
      } else if constexpr (QT == kQBF16) {
        v = bf16_bits_to_f32(((const uint16_t*)p.q)[pc * p.stride + t]);
      } else {
        const f32x2_t c2 = __builtin_amdgcn_cvt_pk_f32_fp8((int)((const uint8_t*)p.q)[pc * p.stride + t], false);
        v = c2[0] * scale[t];
      }
      accumulate<DO>(v - mean[t], bt + t * d, d, acc);
    }
  }
  if (px < p.n_pix)
#pragma unroll
    for (int i = 0; i < DO; ++i)
      if (i < d) p.out[px * d + i] = acc[i];
}

template <int QT, bool VEC>
hipError_t go_proj(const ProjParams& p, const float* bt, const float* mean, const float* scale, dim3 grid,
                   hipStream_t s) {
  if (p.d <= 16) hipLaunchKernelGGL((pca_project_kernel<QT, VEC, 16>), grid, dim3(256), 0, s, p, bt, mean, scale);
  else if (p.d <= 32) hipLaunchKernelGGL((pca_project_kernel<QT, VEC, 32>), grid, dim3(256), 0, s, p, bt, mean, scale);
  else hipLaunchKernelGGL((pca_project_kernel<QT, VEC, 64>), grid, dim3(256), 0, s, p, bt, mean, scale);
  return hipGetLastError();
}

// BF16 maps with rows of whole 32-element groups: the contraction on the
// matrix cores.  Each FP32 basis value is split exactly into three BF16 terms
// (8 + 8 + 8 significand bits), so every product of a BF16 element with a
// term is exact and the only rounding is the FP32 accumulation (about 3D
// additions per output); the centring is applied afterwards,
// out = sum_t q_t b_t - sum_t m_t b_t, with the second sum from the host in
// FP64.  The basis fragments of all groups sit in LDS (the block is
// persistent); a wave takes 64 pixels (4 MFMA column blocks), and each lane
// requests its pixels' groups four steps ahead.
struct PMParams {
  const uint16_t* q;
  int64_t stride, n_pix, n_tiles;
  int steps, d;
  const uint4* frag;            // [steps][3][RB][64 lanes] basis fragments
  const float* mb;              // [d] mean . basis
  float* out;
};

template <int RB>
__global__ __launch_bounds__(512) void pca_mfma_kernel(PMParams p) {
  extern __shared__ uint4 fs[];
  const int nfr = p.steps * 3 * RB * 64;
  for (int i = threadIdx.x; i < nfr; i += 512) fs[i] = p.frag[i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n = lane & 15, g = lane >> 4;
  for (int64_t tile = blockIdx.x; tile < p.n_tiles; tile += gridDim.x) {
    int64_t px[4];
    const uint16_t* row[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      px[nb] = tile * 512 + wave * 64 + 16 * nb + n;
      const int64_t pc = px[nb] < p.n_pix ? px[nb] : p.n_pix - 1;
      row[nb] = p.q + pc * p.stride + 8 * g;
    }
    f32x4_t acc[RB][4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) acc[rb][nb] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    auto load = [&](int st, uint4 (&v)[4]) {
      const int sc = st < p.steps ? st : p.steps - 1;    // clamped: always a valid request
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) v[nb] = *(const uint4*)(row[nb] + 32 * sc);
    };
    auto compute = [&](int st, const uint4 (&v)[4]) {
#pragma unroll
      for (int term = 0; term < 3; ++term)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const uint4 a = fs[((st * 3 + term) * RB + rb) * 64 + lane];
#pragma unroll
          for (int nb = 0; nb < 4; ++nb) acc[rb][nb] = mfma_bf16(a, v[nb], acc[rb][nb]);
        }
    };
    // four steps of query elements in flight
    uint4 qa[4], qb[4], qc[4], qd[4];
    load(0, qa);
    load(1, qb);
    load(2, qc);
    load(3, qd);
    for (int st = 0; st < p.steps; st += 4) {
      compute(st, qa);
      load(st + 4, qa);
      if (st + 1 < p.steps) compute(st + 1, qb);
      load(st + 5, qb);
      if (st + 2 < p.steps) compute(st + 2, qc);
      load(st + 6, qc);
      if (st + 3 < p.steps) compute(st + 3, qd);
      load(st + 7, qd);
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * rb + 4 * g + r;
          if (i < p.d && px[nb] < p.n_pix) p.out[px[nb] * p.d + i] = acc[rb][nb][r] - p.mb[i];
        }
  }
}

}  // namespace

size_t pca_mfma_lds(int D, int d) { return (size_t)(D / 32) * 3 * ((d + 15) / 16) * 64 * 16; }

hipError_t launch_pca_mfma(const uint16_t* q, int64_t stride, int H, int W, int D, const uint4* frag,
                           const float* mb, int d, float* out, int n_cu, hipStream_t s) {
  PMParams p{};
  p.q = q;
  p.stride = stride;
  p.n_pix = (int64_t)H * W;
  p.n_tiles = (p.n_pix + 511) / 512;
  p.steps = D / 32;
  p.d = d;
  p.frag = frag;
  p.mb = mb;
  p.out = out;
  const size_t lds = pca_mfma_lds(D, d);
  const dim3 grid((unsigned)std::min<int64_t>(p.n_tiles, n_cu));
  auto go = [&](auto kern) -> hipError_t {
    if (lds > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, grid, dim3(512), lds, s, p);
    return hipGetLastError();
  };
  timing_begin(K_PCA_PROJECT);
  hipError_t e;
  const int rb = (d + 15) / 16;
  if (rb == 1) e = go(pca_mfma_kernel<1>);
  else if (rb == 2) e = go(pca_mfma_kernel<2>);
  else if (rb == 3) e = go(pca_mfma_kernel<3>);
  else e = go(pca_mfma_kernel<4>);
  timing_end(K_PCA_PROJECT);
  return e;
}

hipError_t launch_pca_project(const void* q, int dtype, int64_t stride, int H, int W, int D, const float* scale,
                              const float* mean, const float* basis_t, int d, float* out, hipStream_t s) {
  ProjParams p{};
  p.q = q;
  p.stride = stride;
  p.n_pix = (int64_t)H * W;
  p.W = W;
  p.H = H;
  p.D = D;
  p.d = d;
  p.out = out;
  const dim3 grid((unsigned)((p.n_pix + 255) / 256));
  const int eb = dtype == VQNNF_F32 ? 4 : dtype == VQNNF_BF16 ? 2 : 1;
  const int al = dtype == VQNNF_FP8_E4M3 ? 8 : 16;
  const bool vec = ((uintptr_t)q % al == 0) && ((stride * eb) % al == 0);
  timing_begin(K_PCA_PROJECT);
  hipError_t e;
  if (dtype == VQNNF_RGB8) e = go_proj<kQRGB8, false>(p, basis_t, mean, scale, grid, s);
  else if (dtype == VQNNF_F32) e = vec ? go_proj<kQF32, true>(p, basis_t, mean, scale, grid, s)
                                       : go_proj<kQF32, false>(p, basis_t, mean, scale, grid, s);
  else if (dtype == VQNNF_BF16) e = vec ? go_proj<kQBF16, true>(p, basis_t, mean, scale, grid, s)
                                        : go_proj<kQBF16, false>(p, basis_t, mean, scale, grid, s);
  else e = vec ? go_proj<kQFP8, true>(p, basis_t, mean, scale, grid, s)
               : go_proj<kQFP8, false>(p, basis_t, mean, scale, grid, s);
  timing_end(K_PCA_PROJECT);
  return e;
}

}  // namespace vqnnf
