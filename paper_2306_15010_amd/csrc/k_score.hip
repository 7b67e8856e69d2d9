// Filter bank + similarity (Sec. 3.2-3.3, eq. 1-2, Alg. 2) + localisation
// (Sec. 4) on gfx950.
//
// For an indicator filter over box [X0,X1) x [Y0,Y1) of the template, the
// window with top-left (x, y) has counts
//   C_j = P[y+Y1][x+X1] - P[y+Y0][x+X1] - P[y+Y1][x+X0] + P[y+Y0][x+X0],
// Alg. 2's dilation filter of a single bin (taps at the bin's corners with
// weights [[1,-1],[-1,1]]).  The score is -sum_f w_f * sum_j |T_f,j - C_f,j|.
// Since a window bin and the template bin have the same area A,
//   sum_j |T_j - C_j| = 2*A - 2*sum_j min(T_j, C_j),
// which lets two channels share one packed 16-bit min and add.
//
// score_fused: the benchmark bank (full window + g x g grid) straight from
// the labels.  A block owns 128 x 16 (or 64 x 16) windows.  For the current window row y
// it keeps, per grid row-band b (rows [y+Y_b, y+Y_b+1)) and per column c of
// the 128 + w - 1 columns it touches, the band's column histogram Q_b[c]
// (uint8 x k in LDS; label values are clamped to the padded channel range
// so an out-of-range label can never address outside LDS).  Moving to row y+1 only changes two labels per band and
// column.  A per-channel prefix along the columns gives
//   H_b[c] = P[y+Y_b+1][x0+c] - P[y+Y_b][x0+c] - (same at column x0),
// the difference of two integral-image rows, and the bin counts of window x
// are H_b[x+X_a+1] - H_b[x+X_a].  The prefix runs over channel chunks so that
// H fits in LDS next to Q.
//
// score_integral: any indicator bank, reading the taps from a precomputed
// integral image (vqnnf_filter's output).
#include "vqnnf_internal.h"

namespace vqnnf {

typedef unsigned short u16x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pk_min_add(uint32_t acc, uint32_t a, uint32_t b) {
  u16x2_t m = __builtin_elementwise_min(__builtin_bit_cast(u16x2_t, a), __builtin_bit_cast(u16x2_t, b));
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2_t, acc) + m);
}

// Orderable key: larger score first, then smaller flat index.
__device__ __forceinline__ unsigned long long best_key(float score, uint32_t idx) {
  uint32_t b = __float_as_uint(score);
  uint32_t o = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  return ((unsigned long long)o << 32) | (unsigned long long)(0xFFFFFFFFu - idx);
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    unsigned long long o = __shfl_xor(v, m);
    v = o > v ? o : v;
  }
  return v;
}

// ================================================================ fused
struct FusedParams {
  const uint8_t* labels;
  int H, W;           // label map
  int w, h;           // template
  int ow, oh;         // heatmap
  int kpad, kc;       // channels (padded) and chunk size
  int qs, hs;         // LDS row strides (dwords) of Q and H
  int nseg, seglen;   // scan segmentation
  int xe[5], ye[5];
  float wt[17];
  int area[17];
  const uint32_t* t16;  // [nf][kpad/2] template counts, u16 pairs
  float* heatmap;
  unsigned long long* best;
};

constexpr int kTYW = 16;    // window rows per tile

// TXW windows per tile row (128 or 64); 256 threads: NP = 256 / TXW threads
// per window, each taking every NP-th channel pair.
template <int G, int TXW>
__global__ __launch_bounds__(256) void score_fused_kernel(FusedParams p) {
  constexpr int NF = 1 + G * G;
  constexpr int NP = 256 / TXW;
  constexpr int kTXW = TXW;
  extern __shared__ uint32_t sm[];
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * kTXW, y0 = blockIdx.y * kTYW;
  const int txv = min(kTXW, p.ow - x0), tyv = min(kTYW, p.oh - y0);
  const int cols = txv + p.w - 1;
  const int kq = p.kpad / 4;
  const int kcp = p.kc / 2, kcq = p.kc / 4;
  uint32_t* Q = sm;                                   // [G][kq][qs]
  uint32_t* Hs = Q + G * kq * p.qs;                   // [G][kcp][hs]
  uint32_t* segt = Hs + G * kcp * p.hs;               // [G][kcq][nseg][2]
  uint32_t* red = segt + G * kcq * p.nseg * 2;        // [NP-1][NF][kTXW]

  // initial band histograms for window row y0
  for (int i = tid; i < G * kq * p.qs; i += 256) Q[i] = 0u;
  __syncthreads();
  for (int c = tid; c < cols; c += 256) {
    for (int b = 0; b < G; ++b) {
      for (int yy = p.ye[b]; yy < p.ye[b + 1]; ++yy) {
        const int l = min((int)p.labels[(int64_t)(y0 + yy) * p.W + x0 + c], p.kpad - 1);
        Q[(b * kq + (l >> 2)) * p.qs + c] += 1u << (8 * (l & 3));
      }
    }
  }

  const int xl = tid % kTXW, half = tid / kTXW;   // half: which 1/NP of the pairs
  for (int dy = 0; dy < tyv; ++dy) {
    const int y = y0 + dy;
    if (dy > 0) {
      for (int c = tid; c < cols; c += 256) {
#pragma unroll
        for (int b = 0; b < G; ++b) {
          const int lo = min((int)p.labels[(int64_t)(y - 1 + p.ye[b]) * p.W + x0 + c], p.kpad - 1);
          const int li = min((int)p.labels[(int64_t)(y - 1 + p.ye[b + 1]) * p.W + x0 + c], p.kpad - 1);
          if (lo != li) {
            Q[(b * kq + (lo >> 2)) * p.qs + c] -= 1u << (8 * (lo & 3));
            Q[(b * kq + (li >> 2)) * p.qs + c] += 1u << (8 * (li & 3));
          }
        }
      }
    }
    __syncthreads();
    uint32_t acc[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] = 0u;

    for (int ch = 0; ch < p.kpad / p.kc; ++ch) {
      // ---- prefix along columns, pass 1: segment-local
      const int items = G * kcq * p.nseg;
      for (int it = tid; it < items; it += 256) {
        const int seg = it % p.nseg, bq = it / p.nseg;
        const int b = bq / kcq, qq = bq % kcq;
        const int c0 = seg * p.seglen, c1 = min(cols, c0 + p.seglen);
        const uint32_t* qrow = Q + (b * kq + ch * kcq + qq) * p.qs;
        uint32_t* h0 = Hs + (b * kcp + 2 * qq) * p.hs;
        uint32_t* h1 = h0 + p.hs;
        uint32_t r0 = 0u, r1 = 0u;
        for (int c = c0; c < c1; ++c) {
          h0[c] = r0;
          h1[c] = r1;
          const uint32_t v = qrow[c];
          r0 += (v & 0xFFu) | ((v & 0xFF00u) << 8);
          r1 += ((v >> 16) & 0xFFu) | ((v >> 8) & 0xFF0000u);
        }
        if (c0 < cols && c1 == cols) {
          h0[cols] = r0;
          h1[cols] = r1;
        }
        segt[(bq * p.nseg + seg) * 2] = r0;
        segt[(bq * p.nseg + seg) * 2 + 1] = r1;
      }
      __syncthreads();
      // ---- pass 2: add the totals of the preceding segments
      for (int it = tid; it < items; it += 256) {
        const int seg = it % p.nseg, bq = it / p.nseg;
        if (seg == 0) continue;
        const int b = bq / kcq, qq = bq % kcq;
        const int c0 = seg * p.seglen, c1 = min(cols, c0 + p.seglen);
        if (c0 >= cols) continue;
        uint32_t o0 = 0u, o1 = 0u;
        for (int s2 = 0; s2 < seg; ++s2) {
          o0 += segt[(bq * p.nseg + s2) * 2];
          o1 += segt[(bq * p.nseg + s2) * 2 + 1];
        }
        uint32_t* h0 = Hs + (b * kcp + 2 * qq) * p.hs;
        uint32_t* h1 = h0 + p.hs;
        const int ce = (c1 == cols) ? cols + 1 : c1;
        for (int c = c0; c < ce; ++c) {
          h0[c] += o0;
          h1[c] += o1;
        }
      }
      __syncthreads();
      // ---- evaluate windows: thread (xl, half) takes every other pair
      if (xl < txv) {
        for (int pl = half; pl < kcp; pl += NP) {
          const int pg = ch * kcp + pl;
          uint32_t full = 0u;
#pragma unroll
          for (int b = 0; b < G; ++b) {
            const uint32_t* hrow = Hs + (b * kcp + pl) * p.hs + xl;
            uint32_t hb[G + 1];
#pragma unroll
            for (int a = 0; a <= G; ++a) hb[a] = hrow[p.xe[a]];
#pragma unroll
            for (int a = 0; a < G; ++a)
              acc[1 + b * G + a] = pk_min_add(acc[1 + b * G + a], hb[a + 1] - hb[a],
                                              p.t16[(1 + b * G + a) * (p.kpad / 2) + pg]);
            full += hb[G] - hb[0];
          }
          acc[0] = pk_min_add(acc[0], full, p.t16[pg]);
        }
      }
      __syncthreads();
    }
    // ---- combine the NP parts, score, localise
    if (half > 0) {
#pragma unroll
      for (int f = 0; f < NF; ++f) red[((half - 1) * NF + f) * kTXW + xl] = acc[f];
    }
    __syncthreads();
    if (half == 0) {
      unsigned long long key = 0ull;
      if (xl < txv) {
        float s = 0.f;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          uint32_t t = acc[f];
#pragma unroll
          for (int q = 1; q < NP; ++q) t += red[((q - 1) * NF + f) * kTXW + xl];
          const int mins = (int)(t & 0xFFFFu) + (int)(t >> 16);
          const int l1 = 2 * p.area[f] - 2 * mins;
          s = fmaf(p.wt[f], (float)l1, s);
        }
        const float score = -s;
        const uint32_t idx = (uint32_t)y * (uint32_t)p.ow + (uint32_t)(x0 + xl);
        p.heatmap[idx] = score;
        key = best_key(score, idx);
      }
      key = wave_max_u64(key);
      if ((tid & 63) == 0 && key) atomicMax(p.best, key);
    }
    __syncthreads();
  }
}

// ================================================================ integral
struct IntParams {
  const int32_t* P;
  int H, W, k, ow, oh, nf;
  const int32_t* boxes;    // [nf][4]
  const int32_t* counts;   // [nf][kpad]
  int kpad;
  const float* weights;
  float* heatmap;
  unsigned long long* best;
};

__global__ __launch_bounds__(256) void score_integral_kernel(IntParams p) {
  const int lane = threadIdx.x & 63;
  const int64_t win = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (win >= (int64_t)p.ow * p.oh) return;
  const int x = (int)(win % p.ow), y = (int)(win / p.ow);
  const int64_t row = (int64_t)(p.W + 1) * p.k;
  float s = 0.f;
  for (int f = 0; f < p.nf; ++f) {
    const int bx0 = p.boxes[4 * f], by0 = p.boxes[4 * f + 1];
    const int bx1 = p.boxes[4 * f + 2], by1 = p.boxes[4 * f + 3];
    const int32_t* p00 = p.P + (int64_t)(y + by0) * row + (int64_t)(x + bx0) * p.k;
    const int32_t* p01 = p.P + (int64_t)(y + by0) * row + (int64_t)(x + bx1) * p.k;
    const int32_t* p10 = p.P + (int64_t)(y + by1) * row + (int64_t)(x + bx0) * p.k;
    const int32_t* p11 = p.P + (int64_t)(y + by1) * row + (int64_t)(x + bx1) * p.k;
    int l1 = 0;
    for (int j = lane; j < p.k; j += 64) {
      const int c = p11[j] - p01[j] - p10[j] + p00[j];
      const int d = p.counts[f * p.kpad + j] - c;
      l1 += d < 0 ? -d : d;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) l1 += __shfl_xor(l1, m);
    s = fmaf(p.weights[f], (float)l1, s);
  }
  if (lane == 0) {
    const float score = -s;
    p.heatmap[win] = score;
    atomicMax(p.best, best_key(score, (uint32_t)win));
  }
}

// ================================================================ launchers
namespace {

struct FusedPlan {
  bool ok;
  int txw, kc, qs, hs, nseg, seglen;
  size_t lds;
};

FusedPlan plan_fused(const DeviceTemplate& t) {
  FusedPlan pl{};
  const int G = t.grid.g;
  int maxband = 0;
  for (int b = 0; b < G; ++b) maxband = std::max(maxband, t.grid.ye[b + 1] - t.grid.ye[b]);
  const int kpad = t.geom.kpad;
  for (int txw = 128; txw >= 64; txw /= 2) {
    const int colsmax = txw + t.w - 1;
    if ((int64_t)maxband * colsmax >= 65536) continue;   // 16-bit prefix would overflow
    const int qs = colsmax | 1, hs = (colsmax + 1) | 1;
    const int np = 256 / txw;
    // chunks need at least one pair per thread part
    for (int kc = kpad; kc >= 2 * np && kc >= 8; kc /= 2) {
      if (kpad % kc) continue;
      int items0 = G * (kc / 4);
      int nseg = std::max(1, 256 / std::max(1, items0));
      int seglen = (colsmax + nseg - 1) / nseg;
      size_t lds = 4 * ((size_t)G * (kpad / 4) * qs + (size_t)G * (kc / 2) * hs +
                        (size_t)G * (kc / 4) * nseg * 2 + (size_t)(np - 1) * (1 + G * G) * txw);
      if (lds <= 160 * 1024) {
        pl.ok = true;
        pl.txw = txw;
        pl.kc = kc;
        pl.qs = qs;
        pl.hs = hs;
        pl.nseg = nseg;
        pl.seglen = seglen;
        pl.lds = lds;
        return pl;
      }
    }
  }
  return pl;
}

template <int G, int TXW>
hipError_t go_fused(const FusedParams& fp, const FusedPlan& pl, hipStream_t s) {
  auto kern = score_fused_kernel<G, TXW>;
  if (pl.lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.lds);
    if (e != hipSuccess) return e;
  }
  dim3 grid((fp.ow + TXW - 1) / TXW, (fp.oh + kTYW - 1) / kTYW);
  hipLaunchKernelGGL(kern, grid, dim3(256), pl.lds, s, fp);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_score_fused(const ScoreArgs& a, hipStream_t s, size_t* lds_bytes_out) {
  const DeviceTemplate& t = *a.t;
  if (!t.grid.valid) return hipErrorInvalidValue;
  FusedPlan pl = plan_fused(t);
  if (!pl.ok) return hipErrorInvalidConfiguration;
  FusedParams fp{};
  fp.labels = a.labels;
  fp.H = a.H;
  fp.W = a.W;
  fp.w = t.w;
  fp.h = t.h;
  fp.ow = a.W - t.w + 1;
  fp.oh = a.H - t.h + 1;
  fp.kpad = t.geom.kpad;
  fp.kc = pl.kc;
  fp.qs = pl.qs;
  fp.hs = pl.hs;
  fp.nseg = pl.nseg;
  fp.seglen = pl.seglen;
  const int G = t.grid.g;
  for (int i = 0; i <= G; ++i) {
    fp.xe[i] = t.grid.xe[i];
    fp.ye[i] = t.grid.ye[i];
  }
  for (int f = 0; f < t.n_filters; ++f) {
    fp.wt[f] = t.weights[f];
    const int32_t* b = &t.boxes[(size_t)f * 4];
    fp.area[f] = (b[2] - b[0]) * (b[3] - b[1]);
  }
  fp.t16 = t.d_counts16;
  fp.heatmap = a.heatmap;
  fp.best = a.best;
  if (lds_bytes_out) *lds_bytes_out = pl.lds;
  timing_begin(K_SCORE_FUSED);
  hipError_t e;
  const bool wide = pl.txw == 128;
  switch (G) {
    case 1: e = wide ? go_fused<1, 128>(fp, pl, s) : go_fused<1, 64>(fp, pl, s); break;
    case 2: e = wide ? go_fused<2, 128>(fp, pl, s) : go_fused<2, 64>(fp, pl, s); break;
    case 3: e = wide ? go_fused<3, 128>(fp, pl, s) : go_fused<3, 64>(fp, pl, s); break;
    case 4: e = wide ? go_fused<4, 128>(fp, pl, s) : go_fused<4, 64>(fp, pl, s); break;
    default: e = hipErrorInvalidValue;
  }
  timing_end(K_SCORE_FUSED);
  return e;
}

bool fused_supported(const DeviceTemplate& t) { return t.grid.valid && plan_fused(t).ok; }

hipError_t launch_score_integral(const ScoreArgs& a, hipStream_t s) {
  const DeviceTemplate& t = *a.t;
  IntParams ip{};
  ip.P = a.P;
  ip.H = a.H;
  ip.W = a.W;
  ip.k = t.k;
  ip.ow = a.W - t.w + 1;
  ip.oh = a.H - t.h + 1;
  ip.nf = t.n_filters;
  ip.boxes = t.d_boxes;
  ip.counts = t.d_counts;
  ip.kpad = t.geom.kpad;
  ip.weights = t.d_weights;
  ip.heatmap = a.heatmap;
  ip.best = a.best;
  const int64_t nwin = (int64_t)ip.ow * ip.oh;
  timing_begin(K_SCORE_INTEGRAL);
  hipLaunchKernelGGL(score_integral_kernel, dim3((unsigned)((nwin + 3) / 4)), dim3(256), 0, s, ip);
  timing_end(K_SCORE_INTEGRAL);
  return hipGetLastError();
}

}  // namespace vqnnf
