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
#include "dev_common.h"

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

// Block-wide maximum of the keys (blockDim.x = 256), then one atomicMax per
// block, skipped when the stored key is already larger: the key only grows,
// so a stale read can only cost an unneeded atomic.
__device__ __forceinline__ void block_max_to(unsigned long long key, unsigned long long* best) {
  __shared__ unsigned long long wmax[4];
  key = wave_max_u64(key);
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = key;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long k = wmax[0];
#pragma unroll
    for (int i = 1; i < 4; ++i) k = wmax[i] > k ? wmax[i] : k;
    if (k > __hip_atomic_load(best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(best, k);
  }
}

// ================================================================ fused
// One block owns a tile of up to kTXW x tyw windows and one group of kKG
// channels.  LDS holds, per grid row-band b and per column c of the
// txw + w - 1 columns the tile touches:
//   Q[b][c]  the band's column histogram (channel pairs as packed u16,
//            four pairs per 16-byte entry),
//   H[b][c]  its prefix along the columns, H[b][c] = sum_{c' < c} Q[b][c'],
// so the count of bin (a, b) of window x is H[b][x + X_{a+1}] - H[b][x + X_a]
// and the full window is the sum of the bands' H[b][x + w] - H[b][x].
// Per window row, two phases separated by barriers:
//   1. one wave per (band, pair group) row rebuilds its prefix: lane s sums
//      segment s (kSL columns, kept in registers), a DPP scan of the segment
//      totals gives the offsets, the lane writes its segment of H;
//   2. every thread scores one window against four channel pairs,
//      accumulating sum_j min(T_j, C_j) with v_dot2_u32_u16, while the
//      column threads move Q down to the next row (two labels per band and
//      column change).
// The integer sums of the group are written per window; a second kernel adds
// the groups, forms eq. 2 and the argmax.
constexpr int kSL = 7;                 // columns per prefix segment (odd: a wave's lanes hit distinct banks)
constexpr int kNSeg = 53;              // segments per row (<= 64 lanes)
constexpr int kHS = kSL * kNSeg;       // LDS row length in 16-byte entries
constexpr int kColsMax = kHS - kSL;    // nseg = cols / kSL + 1 segments cover [0, cols]
constexpr int kKG = 16;                // channels per block
constexpr int kPQ = kKG / 8;           // 16-byte entries (four pairs) per column per band
constexpr int kTXW = 256;              // windows per tile row
constexpr int kST = 512;               // threads per block: kTXW windows x kPQ pair groups

struct TileParams {
  const uint8_t* labels;
  int H, W;           // label map
  int w, h;           // template
  int ow, oh;         // heatmap
  int txw, tyw;       // windows per tile row (<= kTXW) and window rows per tile
  int kpad;
  int xe[5], ye[5];
  const uint32_t* t16;  // [nf][kpad/2] template counts, u16 pairs
  uint32_t* part;       // [n_groups][nacc][pstride] sums of min(T_j, C_j)
  int64_t pstride;      // windows per partial row, oh*ow rounded up to 4
};

typedef unsigned long long u64x2_t __attribute__((ext_vector_type(2)));

// Four packed pairs added as two 64-bit words: every 16-bit count stays below
// 2^16, so no carry crosses a field.
__device__ __forceinline__ uint4 add4(uint4 a, uint4 b) {
  return __builtin_bit_cast(uint4, __builtin_bit_cast(u64x2_t, a) + __builtin_bit_cast(u64x2_t, b));
}
__device__ __forceinline__ uint32_t comp(uint4 v, int s) {
  return s == 0 ? v.x : s == 1 ? v.y : s == 2 ? v.z : v.w;
}
__device__ __forceinline__ uint32_t min_dot(uint32_t c, uint32_t t, uint32_t acc) {
  const u16x2_t m = __builtin_elementwise_min(__builtin_bit_cast(u16x2_t, c), __builtin_bit_cast(u16x2_t, t));
  return __builtin_amdgcn_udot2(m, (u16x2_t){1, 1}, acc, false);
}

// UNI: every bin has the same weight, so the bins share one accumulator
// (accumulator 0: full window, 1: bins); otherwise one per filter.
template <int G, bool UNI>
__global__ __launch_bounds__(kST) void score_tile_kernel(TileParams p) {
  constexpr int NF = 1 + G * G;
  constexpr int NACC = UNI ? 2 : NF;
  constexpr int NR = G * kPQ;                        // (band, pair group) rows
  static_assert(NR <= kST / 64, "one wave per prefix row");
  __shared__ uint4 Qs[NR][kHS];
  __shared__ uint4 Hs[NR][kHS];
  __shared__ uint32_t red[NACC][kTXW];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int x0 = blockIdx.x * p.txw, y0 = blockIdx.y * p.tyw;
  const int grp = blockIdx.z, j0 = grp * kKG;
  const int txv = min(p.txw, p.ow - x0), tyv = min(p.tyw, p.oh - y0);
  const int cols = txv + p.w - 1;
  const int nseg = cols / kSL + 1;                   // segments cover [0, cols]
  uint32_t* Q32 = (uint32_t*)&Qs[0][0];
  // channel jl of the group lives in row b*kPQ + jl/8, word (jl/2)%4, half jl%2
  auto qword = [&](int b, int jl, int c) -> uint32_t* {
    return Q32 + ((b * kPQ + (jl >> 3)) * kHS + c) * 4 + ((jl >> 1) & 3);
  };

  for (int i = tid; i < NR * kHS; i += kST) (&Qs[0][0])[i] = make_uint4(0u, 0u, 0u, 0u);
  __syncthreads();
  // band histograms at the tile's first row: items of 8 rows of one column,
  // the 8 label loads issued together
  const int nrc = (p.h + 7) / 8;
  for (int i = tid; i < nrc * cols; i += kST) {
    const int c = i % cols, r0 = (i / cols) * 8;
    int l8[8];
#pragma unroll
    for (int r = 0; r < 8; ++r)
      l8[r] = (r0 + r < p.h) ? (int)p.labels[(int64_t)(y0 + r0 + r) * p.W + x0 + c] - j0 : -1;
    int b = 0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if (r0 + r >= p.h) break;
      while (r0 + r >= p.ye[b + 1]) ++b;
      if ((unsigned)l8[r] < (unsigned)kKG) atomicAdd(qword(b, l8[r], c), 1u << (16 * (l8[r] & 1)));
    }
  }

  // scoring role: window xl of the tile, pair group pq (uniform per wave)
  const int pq = wv & 1;
  const int xl = (wv >> 1) * 64 + lane;
  uint32_t T[NF][4];
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int s = 0; s < 4; ++s) T[f][s] = p.t16[f * (p.kpad / 2) + j0 / 2 + pq * 4 + s];
  // labels leaving / entering each band at the next row step, prefetched
  int lo[G], li[G];
  auto fetch = [&](int ynext, int c) {
#pragma unroll
    for (int b = 0; b < G; ++b) {
      lo[b] = (int)p.labels[(int64_t)(ynext - 1 + p.ye[b]) * p.W + x0 + c] - j0;
      li[b] = (int)p.labels[(int64_t)(ynext - 1 + p.ye[b + 1]) * p.W + x0 + c] - j0;
    }
  };
  if (tyv > 1 && tid < cols) fetch(y0 + 1, tid);

  uint32_t acc[NACC];
  auto store_row = [&](int yy) {  // pair group 0 adds group 1's sums
    const int64_t win = (int64_t)yy * p.ow + x0 + xl;
#pragma unroll
    for (int a = 0; a < NACC; ++a) p.part[((int64_t)grp * NACC + a) * p.pstride + win] = acc[a] + red[a][xl];
  };
  for (int dy = 0; dy < tyv; ++dy) {
    const int y = y0 + dy;
    __syncthreads();   // Q at row y complete; previous row's H and red consumed
    // ---- phase 1: prefix of row wv, lane = segment
    if (wv < NR) {
      const int c0 = lane * kSL;
      const bool act = lane < nseg;
      uint4 loc[kSL];
      uint4 run = make_uint4(0u, 0u, 0u, 0u);
      if (act) {
#pragma unroll
        for (int i = 0; i < kSL; ++i) {
          loc[i] = run;
          run = add4(run, Qs[wv][c0 + i]);
        }
      }
      const uint4 inc = make_uint4(wave_incl_scan(run.x), wave_incl_scan(run.y), wave_incl_scan(run.z),
                                   wave_incl_scan(run.w));
      const uint4 off = make_uint4(inc.x - run.x, inc.y - run.y, inc.z - run.z, inc.w - run.w);
      if (act) {
#pragma unroll
        for (int i = 0; i < kSL; ++i) Hs[wv][c0 + i] = add4(off, loc[i]);
      }
    }
    if (dy > 0 && pq == 0 && xl < txv) store_row(y - 1);
    __syncthreads();   // H at row y complete
    // ---- phase 2: score window xl against pairs 4*pq .. 4*pq + 3 of the group
#pragma unroll
    for (int a = 0; a < NACC; ++a) acc[a] = 0u;
    if (xl < txv) {
      uint32_t full[4] = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int b = 0; b < G; ++b) {
        uint4 hv[G + 1];
#pragma unroll
        for (int a = 0; a <= G; ++a) hv[a] = Hs[b * kPQ + pq][xl + p.xe[a]];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
          for (int a = 0; a < G; ++a) {
            const uint32_t bin = comp(hv[a + 1], s) - comp(hv[a], s);
            const int ai = UNI ? 1 : 1 + b * G + a;
            acc[ai] = min_dot(bin, T[1 + b * G + a][s], acc[ai]);
          }
          full[s] += comp(hv[G], s) - comp(hv[0], s);
        }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) acc[0] = min_dot(full[s], T[0][s], acc[0]);
      if (pq == 1) {
#pragma unroll
        for (int a = 0; a < NACC; ++a) red[a][xl] = acc[a];
      }
    }
    // ---- vertical update of Q to row y + 1, then prefetch for row y + 2
    if (dy + 1 < tyv && tid < cols) {
      const int c = tid;
#pragma unroll
      for (int b = 0; b < G; ++b) {
        if (lo[b] == li[b]) continue;
        if ((unsigned)lo[b] < (unsigned)kKG) atomicSub(qword(b, lo[b], c), 1u << (16 * (lo[b] & 1)));
        if ((unsigned)li[b] < (unsigned)kKG) atomicAdd(qword(b, li[b], c), 1u << (16 * (li[b] & 1)));
      }
      if (dy + 2 < tyv) fetch(y + 2, c);
    }
  }
  __syncthreads();
  if (pq == 0 && xl < txv) store_row(y0 + tyv - 1);
}

// Adds the groups' integer sums, forms eq. 2 and the argmax.
struct CombineParams {
  const uint32_t* part;
  int64_t nwin, pstride;
  bool vec_out;       // heatmap 16-byte aligned
  int ngroups;
  float wt[17];       // per accumulator weight
  int area2[17];      // per accumulator: twice the summed bin areas
  float* heatmap;
  unsigned long long* best;
};

// Four consecutive windows per thread: 16-byte loads of every partial row
// (rows are padded to a multiple of four windows).
template <int NACC>
__global__ __launch_bounds__(256) void score_combine_kernel(CombineParams p) {
  const int64_t w0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  unsigned long long key = 0ull;
  if (w0 < p.nwin) {
    uint4 m[NACC];
#pragma unroll
    for (int a = 0; a < NACC; ++a) m[a] = make_uint4(0u, 0u, 0u, 0u);
    for (int g = 0; g < p.ngroups; ++g) {
      uint4 v[NACC];
#pragma unroll
      for (int a = 0; a < NACC; ++a) v[a] = *(const uint4*)(p.part + ((int64_t)g * NACC + a) * p.pstride + w0);
#pragma unroll
      for (int a = 0; a < NACC; ++a)
        m[a] = make_uint4(m[a].x + v[a].x, m[a].y + v[a].y, m[a].z + v[a].z, m[a].w + v[a].w);
    }
    // sum_j |T_j - C_j| = 2A - 2 sum_j min(T_j, C_j), exact in integers
    float sc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float s = 0.f;
#pragma unroll
      for (int a = 0; a < NACC; ++a) {
        const uint32_t mi = i == 0 ? m[a].x : i == 1 ? m[a].y : i == 2 ? m[a].z : m[a].w;
        s = fmaf(p.wt[a], (float)(p.area2[a] - 2 * (int)mi), s);
      }
      sc[i] = -s;
    }
    const int nv = (int)min((int64_t)4, p.nwin - w0);
    if (nv == 4 && p.vec_out) {
      *(float4*)(p.heatmap + w0) = make_float4(sc[0], sc[1], sc[2], sc[3]);
    } else {
      for (int i = 0; i < nv; ++i) p.heatmap[w0 + i] = sc[i];
    }
    for (int i = 0; i < nv; ++i) {
      const unsigned long long k2 = best_key(sc[i], (uint32_t)(w0 + i));
      key = k2 > key ? k2 : key;
    }
  }
  block_max_to(key, p.best);
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
  unsigned long long key = 0ull;
  if (win < (int64_t)p.ow * p.oh) {  // uniform per wave
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
      key = best_key(score, (uint32_t)win);
    }
  }
  block_max_to(key, p.best);
}

// ================================================================ launchers
namespace {

struct TilePlan {
  bool ok;
  bool uni;
  int txw, tyw;
  int nacc;
};

// Tiles are as wide as the LDS rows allow (at most kTXW windows, at least 32).
TilePlan plan_tile(const DeviceTemplate& t) {
  TilePlan pl{};
  if (!t.grid.valid) return pl;
  const int G = t.grid.g;
  if (G < 1 || G > 4 || t.geom.kpad % kKG) return pl;
  int maxband = 0;
  for (int b = 0; b < G; ++b) maxband = std::max(maxband, t.grid.ye[b + 1] - t.grid.ye[b]);
  pl.txw = std::min(kTXW, kColsMax + 1 - t.w);
  if (pl.txw < 32) return pl;
  if ((int64_t)maxband * (kColsMax + 1) >= 65536) return pl;   // u16 prefix counts
  pl.uni = true;
  for (int f = 2; f < t.n_filters; ++f)
    if (t.weights[f] != t.weights[1]) pl.uni = false;
  pl.nacc = pl.uni ? 2 : t.n_filters;
  pl.tyw = 32;
  pl.ok = true;
  return pl;
}

template <int G, bool UNI>
hipError_t go_tile(const TileParams& tp, hipStream_t s) {
  dim3 grid((tp.ow + tp.txw - 1) / tp.txw, (tp.oh + tp.tyw - 1) / tp.tyw, tp.kpad / kKG);
  hipLaunchKernelGGL((score_tile_kernel<G, UNI>), grid, dim3(kST), 0, s, tp);
  return hipGetLastError();
}

template <int G>
hipError_t go_tile_u(const TileParams& tp, bool uni, hipStream_t s) {
  return uni ? go_tile<G, true>(tp, s) : go_tile<G, false>(tp, s);
}

hipError_t go_combine(const CombineParams& cp, int nacc, hipStream_t s) {
  const dim3 grid((unsigned)((cp.nwin + 1023) / 1024)), blk(256);
  switch (nacc) {
    case 2: hipLaunchKernelGGL((score_combine_kernel<2>), grid, blk, 0, s, cp); break;
    case 5: hipLaunchKernelGGL((score_combine_kernel<5>), grid, blk, 0, s, cp); break;
    case 10: hipLaunchKernelGGL((score_combine_kernel<10>), grid, blk, 0, s, cp); break;
    case 17: hipLaunchKernelGGL((score_combine_kernel<17>), grid, blk, 0, s, cp); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

size_t fused_partial_bytes(const DeviceTemplate& t, int H, int W) {
  TilePlan pl = plan_tile(t);
  if (!pl.ok) return 0;
  const int64_t nwin = (int64_t)(H - t.h + 1) * (W - t.w + 1);
  return (size_t)(t.geom.kpad / kKG) * pl.nacc * ((nwin + 3) / 4 * 4) * 4;
}

hipError_t launch_score_fused(const ScoreArgs& a, hipStream_t s, size_t* lds_bytes_out) {
  const DeviceTemplate& t = *a.t;
  const int ow = a.W - t.w + 1, oh = a.H - t.h + 1;
  if (!t.grid.valid || !a.partials) return hipErrorInvalidValue;
  TilePlan pl = plan_tile(t);
  if (!pl.ok) return hipErrorInvalidConfiguration;
  // equal tile widths; tile height from the caller (autotuned) or the default
  const int nx = (ow + pl.txw - 1) / pl.txw;
  pl.txw = (ow + nx - 1) / nx;
  pl.tyw = a.tyw > 0 ? std::min(a.tyw, oh) : fused_default_tyw(t, a.H, a.W, a.n_cu);
  TileParams tp{};
  tp.labels = a.labels;
  tp.H = a.H;
  tp.W = a.W;
  tp.w = t.w;
  tp.h = t.h;
  tp.ow = ow;
  tp.oh = oh;
  tp.txw = pl.txw;
  tp.tyw = pl.tyw;
  tp.kpad = t.geom.kpad;
  const int G = t.grid.g;
  for (int i = 0; i <= G; ++i) {
    tp.xe[i] = t.grid.xe[i];
    tp.ye[i] = t.grid.ye[i];
  }
  tp.t16 = t.d_counts16;
  tp.part = (uint32_t*)a.partials;
  tp.pstride = ((int64_t)ow * oh + 3) / 4 * 4;
  if (lds_bytes_out) {
    const int NR = G * kPQ;
    *lds_bytes_out = (size_t)2 * NR * kHS * 16 + (size_t)pl.nacc * kTXW * 4;
  }
  timing_begin(K_SCORE_FUSED);
  hipError_t e;
  switch (G) {
    case 1: e = go_tile_u<1>(tp, pl.uni, s); break;
    case 2: e = go_tile_u<2>(tp, pl.uni, s); break;
    case 3: e = go_tile_u<3>(tp, pl.uni, s); break;
    case 4: e = go_tile_u<4>(tp, pl.uni, s); break;
    default: e = hipErrorInvalidValue;
  }
  timing_end(K_SCORE_FUSED);
  if (e != hipSuccess) return e;
  CombineParams cp{};
  cp.part = tp.part;
  cp.nwin = (int64_t)ow * oh;
  cp.pstride = tp.pstride;
  cp.vec_out = ((uintptr_t)a.heatmap % 16) == 0;
  cp.ngroups = tp.kpad / kKG;
  // accumulator a covers filters: UNI -> {0}, {1..NF-1}; else {a}
  for (int f = 0; f < t.n_filters; ++f) {
    const int32_t* b = &t.boxes[(size_t)f * 4];
    const int area = (b[2] - b[0]) * (b[3] - b[1]);
    const int ai = pl.uni ? (f == 0 ? 0 : 1) : f;
    cp.wt[ai] = t.weights[f];
    cp.area2[ai] += 2 * area;
  }
  cp.heatmap = a.heatmap;
  cp.best = a.best;
  timing_begin(K_SCORE_COMBINE);
  e = go_combine(cp, pl.nacc, s);
  timing_end(K_SCORE_COMBINE);
  return e;
}

bool fused_supported(const DeviceTemplate& t) { return plan_tile(t).ok; }

// Tiles fill whole rounds of two blocks per compute unit (at least 8 rows).
int fused_default_tyw(const DeviceTemplate& t, int H, int W, int n_cu) {
  TilePlan pl = plan_tile(t);
  const int ow = W - t.w + 1, oh = H - t.h + 1;
  const int nx = (ow + pl.txw - 1) / std::max(pl.txw, 1);
  const int per_row = nx * (t.geom.kpad / kKG);
  const int slots = 2 * std::max(n_cu, 1);
  const int ny = std::max(1, (slots + per_row - 1) / per_row);
  return std::min(std::max(8, (oh + ny - 1) / ny), std::max(oh, 1));
}

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
