// Filter bank + similarity (Sec. 3.2-3.3, eq. 1-2, Alg. 2) + localisation
// (Sec. 4) on gfx950.
//
// For an indicator filter over box [X0,X1) x [Y0,Y1) of the template, the
// window with top-left (x, y) has counts
//   C_j = P[y+Y1][x+X1] - P[y+Y0][x+X1] - P[y+Y1][x+X0] + P[y+Y0][x+X0],
// Alg. 2's dilation filter of a single bin (taps at the bin's corners with
// weights [[1,-1],[-1,1]]).  The score is -sum_f w_f * sum_j |T_f,j - C_f,j|,
// summed two channels at a time with v_sad_u16 (or, where twice a filter
// area overflows 16 bits, as 2*A - 2*sum_j min(T_j, C_j), since a window bin
// and the template bin have the same area A).
//
// score_fused: the benchmark bank (full window + g x g grid) straight from
// the labels, tile by tile (below): per grid row-band b and column c the
// band's column histogram Q_b[c] and its prefix along the columns
//   H_b[c] = P[y+Y_b+1][x0+c] - P[y+Y_b][x0+c] - (same at column x0),
// the difference of two integral-image rows, so the bin counts of window x
// are H_b[x+X_a+1] - H_b[x+X_a].  Moving to window row y+1 changes two
// labels per band and column.
//
// score_integral: any indicator bank, reading the taps from a precomputed
// integral image (vqnnf_filter's output).
#include "vqnnf_internal.h"

#include <algorithm>
#include <cstring>
#include <vector>
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
// One block owns a tile of up to kTXW x tyw windows and one group of KG
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
//   2. every thread scores one window against four channel pairs and hands
//      its sums to LDS, while the column threads move Q down to the next row
//      (two labels per band and column change).
// The previous row's sums are added over the pair groups and stored during
// phase 1 by the waves that have no prefix row.  Bins of equal weight share
// one sum.  With one channel group the tile kernel forms eq. 2 and the
// argmax itself; otherwise the integer sums of the group are written per
// window as 16-bit words (at most twice the window area, kept below 2^16)
// and a second kernel adds the groups, forms eq. 2 and the argmax.
constexpr int kSL = 7;                 // columns per prefix segment (odd: a wave's lanes hit distinct banks)
constexpr int kNSeg = 53;              // segments per row (<= 64 lanes)
constexpr int kHS = kSL * kNSeg;       // LDS row length in 16-byte entries
constexpr int kColsMax = kHS - kSL;    // nseg = cols / kSL + 1 segments cover [0, cols]
// Channels per block (KG, a template parameter): 32 (four pair groups, 1024
// threads) where the grid has at most 3 x 3 bins and k pads to a multiple of
// 32, else 16 (two pair groups, 512 threads); KG / 8 16-byte entries (four
// pairs each) per column per band.  Wider blocks re-prime their histograms
// and rebuild their prefixes for more channels at once.
constexpr int kTXW = 256;              // windows per tile row
constexpr int kMaxCls = 4;             // bin weight classes (distinct bin weights)
constexpr int kMaxAcc = 1 + kMaxCls;   // stored sums per window: full window + classes

struct TileParams {
  const uint8_t* labels;
  int H, W;           // label map
  int w, h;           // template
  int ow, oh;         // heatmap
  int txw, tyw;       // windows per tile row (<= kTXW) and window rows per tile
  int kpad;
  int xe[5], ye[5];
  const uint32_t* t16;  // [nf][kpad/2] template counts, u16 pairs
  uint16_t* part;       // [ng][nacc][pstride] sums of min(T_j, C_j)
  int64_t pstride;      // windows per partial row, oh*ow rounded up to 4
  int nacc;             // sums per window: 1 + weight classes of the bins
  uint32_t cmask[kMaxCls];  // bit f of cmask[c - 1]: bin filter f in sum c (unused: 0)
  int nx, ng;           // tiles per heatmap row, channel groups
  uint32_t b0;          // batched launches: first block of the pair
  // one channel group: eq. 2 per sum a, the heatmap and the best key
  float wt[kMaxAcc];
  // sum a's L1 term sum_j |T_j - C_j| = area2[a] + cmul[a] * (stored sum):
  // (0, 1) for sums of |T_j - C_j|, (twice the filters' area, -2) for sums
  // of min(T_j, C_j)
  int area2[kMaxAcc];
  int cmul[kMaxAcc];
  float* heatmap;
  unsigned long long* best;
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

// Block-wide maximum of the keys for blocks of NW waves, then one atomicMax.
template <int NW>
__device__ __forceinline__ void block_max_n(unsigned long long key, unsigned long long* best) {
  __shared__ unsigned long long wmax[NW];
  key = wave_max_u64(key);
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = key;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long k = wmax[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) k = wmax[i] > k ? wmax[i] : k;
    if (k > __hip_atomic_load(best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(best, k);
  }
}

// Pointers read from an argument table are generic; the kernels only touch
// global memory through them, which lets them use global (not flat) accesses.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gbl(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// UNI: every bin has the same weight, so the bins share one accumulator
// (accumulator 0: full window, 1: bins); otherwise one per filter while
// scoring, merged into the stored sums at the end of each row.
// SAD: the accumulators sum |T_j - C_j| (v_sad_u16: two channels per
// instruction, one instruction per channel pair and bin); otherwise
// min(T_j, C_j) (v_pk_min_u16 + v_dot2_u32_u16), whose sums stay below the
// window area where twice the area overflows 16 bits.
template <int G, bool UNI, int KG, bool SAD>
__device__ __forceinline__ void score_tile_body(const TileParams& p, int bx, int by, int grp) {
  constexpr int kPQ = KG / 8;                        // pair groups
  constexpr int kST = kTXW * kPQ;                    // threads
  constexpr int NF = 1 + G * G;
  constexpr int NACC = UNI ? 2 : NF;                 // accumulators while scoring
  constexpr int NOUT = UNI ? 2 : 1 + kMaxCls;        // sums after merging bins of equal weight
  constexpr int NR = G * kPQ;                        // (band, pair group) rows
  static_assert(NR <= kST / 64, "one wave per prefix row");
  static_assert(kColsMax + 1 <= kST, "one column per thread");
  __shared__ uint4 Qs[NR][kHS];
  __shared__ uint4 Hs[NR][kHS];
  __shared__ uint16_t red[kPQ][NOUT][kTXW];          // every pair group's sums of the row (< 2^16)
  const auto labs = gbl(p.labels);
  const auto t16 = gbl(p.t16);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int x0 = bx * p.txw, y0 = by * p.tyw;
  const int j0 = grp * KG;
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
  // four items per thread at a time with their 32 label loads issued together
  const int nrc = (p.h + 7) / 8;
  const int nit = nrc * cols;
  constexpr int kPI = 4;
  for (int i0 = tid; i0 < nit; i0 += kPI * kST) {
    int l8[kPI][8];
#pragma unroll
    for (int u = 0; u < kPI; ++u) {
      const int i = i0 + u * kST;
      const int c = i % cols, r0 = (i / cols) * 8;
#pragma unroll
      for (int r = 0; r < 8; ++r)
        l8[u][r] = (i < nit && r0 + r < p.h) ? (int)labs[(int64_t)(y0 + r0 + r) * p.W + x0 + c] : -1;
    }
#pragma unroll
    for (int u = 0; u < kPI; ++u) {
      const int i = i0 + u * kST;
      if (i >= nit) break;
      const int c = i % cols, r0 = (i / cols) * 8;
      int b = 0;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        if (r0 + r >= p.h) break;
        while (r0 + r >= p.ye[b + 1]) ++b;
        const int l = l8[u][r] - j0;
        if ((unsigned)l < (unsigned)KG) atomicAdd(qword(b, l, c), 1u << (16 * (l & 1)));
      }
    }
  }

  // scoring role: window xl of the tile, pair group pq (uniform per wave)
  const int pq = wv & (kPQ - 1);
  const int xl = (wv / kPQ) * 64 + lane;
  uint32_t T[NF][4];
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int s = 0; s < 4; ++s) T[f][s] = t16[f * (p.kpad / 2) + j0 / 2 + pq * 4 + s];
  // labels leaving / entering each band at the next row step, prefetched a
  // step ahead; kept as loaded (the group offset is taken at use), so the
  // loads stay in flight across the barriers until the next step needs them
  int lo[G], li[G];
  auto fetch = [&](int ynext, int c) {
#pragma unroll
    for (int b = 0; b < G; ++b) {
      lo[b] = (int)labs[(int64_t)(ynext - 1 + p.ye[b]) * p.W + x0 + c];
      li[b] = (int)labs[(int64_t)(ynext - 1 + p.ye[b + 1]) * p.W + x0 + c];
    }
  };
  if (tyv > 1 && tid < cols) fetch(y0 + 1, tid);

  uint32_t acc[NACC];
  unsigned long long key = 0ull;
  // one channel pair's term of a bin (packed counts c, template counts t)
  auto term = [](uint32_t c, uint32_t t, uint32_t a) -> uint32_t {
    if constexpr (SAD) return __builtin_amdgcn_sad_u16(c, t, a);
    else return min_dot(c, t, a);
  };
  // the stored sums: full window, then the bins of each weight class
  auto merge = [&](uint32_t (&o)[NOUT]) {
    if constexpr (UNI) {
      o[0] = acc[0];
      o[1] = acc[1];
    } else {
      o[0] = acc[0];
#pragma unroll
      for (int c = 1; c < NOUT; ++c) {
        const uint32_t cm = p.cmask[c - 1];
        uint32_t v = 0u;
#pragma unroll
        for (int f = 1; f < NF; ++f) v += ((cm >> f) & 1u) ? acc[f] : 0u;
        o[c] = v;
      }
    }
  };
  // window x of row yy: adds the pair groups' sums from LDS and stores them,
  // or with one channel group forms the score itself
  auto store_one = [&](int yy, int x) {
    uint32_t v[NOUT];
#pragma unroll
    for (int a = 0; a < NOUT; ++a) v[a] = red[0][a][x];
#pragma unroll
    for (int g2 = 1; g2 < kPQ; ++g2)
#pragma unroll
      for (int a = 0; a < NOUT; ++a) v[a] += red[g2][a][x];
    const int64_t win = (int64_t)yy * p.ow + x0 + x;
    float s = 0.f;
#pragma unroll
    for (int a = 0; a < NOUT; ++a) {
      if (a >= p.nacc) break;
      const uint32_t o = v[a];
      if (p.ng == 1) {
        s = fmaf(p.wt[a], (float)(p.area2[a] + p.cmul[a] * (int)o), s);
      } else {
        gbl(p.part)[((int64_t)grp * p.nacc + a) * p.pstride + win] = (uint16_t)o;
      }
    }
    if (p.ng == 1) {
      const float sc = -s;
      gbl(p.heatmap)[win] = sc;
      const unsigned long long k2 = best_key(sc, (uint32_t)win);
      key = k2 > key ? k2 : key;
    }
  };
  // the row's stores go to the waves without a prefix row (they are idle
  // while the prefix rows are rebuilt), or to every wave when all have one
  constexpr int NW = kST / 64;
  constexpr int SW = NW > NR ? NR : 0;               // first storing wave
  auto store_row = [&](int yy) {
    for (int x = tid - SW * 64; x >= 0 && x < txv; x += kST - SW * 64) store_one(yy, x);
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
    if (dy > 0) store_row(y - 1);
    __syncthreads();   // H at row y complete
    // ---- phase 2: score window xl against pairs 4*pq .. 4*pq + 3 of the group
#pragma unroll
    for (int a = 0; a < NACC; ++a) acc[a] = 0u;
    if (xl < txv) {
      uint32_t full[4] = {0u, 0u, 0u, 0u};
      // uniform bins: one sum per channel pair, added at the end, so the
      // G*G*4 terms form four independent chains instead of one
      uint32_t bins[4] = {0u, 0u, 0u, 0u};
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
            if constexpr (UNI) {
              bins[s] = term(bin, T[1 + b * G + a][s], bins[s]);
            } else {
              const int ai = 1 + b * G + a;
              acc[ai] = term(bin, T[1 + b * G + a][s], acc[ai]);
            }
          }
          full[s] += comp(hv[G], s) - comp(hv[0], s);
        }
      }
      if constexpr (UNI) acc[1] = (bins[0] + bins[1]) + (bins[2] + bins[3]);
      uint32_t f01 = term(full[0], T[0][0], 0u), f23 = term(full[2], T[0][2], 0u);
      f01 = term(full[1], T[0][1], f01);
      f23 = term(full[3], T[0][3], f23);
      acc[0] = f01 + f23;
      uint32_t o[NOUT];
      merge(o);
#pragma unroll
      for (int a = 0; a < NOUT; ++a) red[pq][a][xl] = (uint16_t)o[a];
    }
    // ---- vertical update of Q to row y + 1, then prefetch for row y + 2
    if (dy + 1 < tyv && tid < cols) {
      const int c = tid;
#pragma unroll
      for (int b = 0; b < G; ++b) {
        if (lo[b] == li[b]) continue;
        const int o = lo[b] - j0, e = li[b] - j0;
        if ((unsigned)o < (unsigned)KG) atomicSub(qword(b, o, c), 1u << (16 * (o & 1)));
        if ((unsigned)e < (unsigned)KG) atomicAdd(qword(b, e, c), 1u << (16 * (e & 1)));
      }
      if (dy + 2 < tyv) fetch(y + 2, c);
    }
  }
  __syncthreads();
  store_row(y0 + tyv - 1);
  if (p.ng == 1) block_max_n<kST / 64>(key, p.best);
}

template <int G, bool UNI, int KG, bool SAD>
__global__ __launch_bounds__(kTXW * (KG / 8)) void score_tile_kernel(TileParams p) {
  score_tile_body<G, UNI, KG, SAD>(p, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Batched: block -> pair from a table, then (group, tile column, tile row)
// with the channel group fastest.
template <int G, bool UNI, int KG, bool SAD>
__global__ __launch_bounds__(kTXW * (KG / 8)) void score_tile_batch_kernel(const TileParams* __restrict__ tab,
                                                                           const uint32_t* __restrict__ blk) {
  const TileParams& p = tab[blk[blockIdx.x]];
  const int b = (int)(blockIdx.x - p.b0);
  const int grp = b % p.ng, t = b / p.ng;
  score_tile_body<G, UNI, KG, SAD>(p, t % p.nx, t / p.nx, grp);
}

typedef unsigned int u32x2_v __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4_v __attribute__((ext_vector_type(4)));
typedef float f32x4_v __attribute__((ext_vector_type(4)));

// Adds the groups' integer sums, forms eq. 2 and the argmax.
struct CombineParams {
  const uint16_t* part;
  int64_t nwin, pstride;
  int vec_out;        // heatmap 16-byte aligned
  int ngroups;
  uint32_t b0;        // batched launches: first block of the pair
  float wt[kMaxAcc];  // per stored sum
  int area2[kMaxAcc]; // per stored sum: L1 term = area2 + cmul * (sum over groups)
  int cmul[kMaxAcc];
  float* heatmap;
  unsigned long long* best;
};

// Two quads of four consecutive windows per thread (a block covers
// kCombineWin windows): 8-byte loads of every partial row (rows are padded
// to a multiple of four windows), issued for several channel groups at a
// time; one best-key update per block.
constexpr int kCombineQ = 2;
constexpr int kCombineWin = 256 * 4 * kCombineQ;

template <int NACC>
__device__ __forceinline__ void combine_body(const CombineParams& p, int64_t blk) {
  constexpr int GB = NACC <= 2 ? 4 : 2;              // channel groups per batch of loads
  unsigned long long key = 0ull;
  int64_t w[kCombineQ];
  uint4 m[kCombineQ][NACC];
#pragma unroll
  for (int q = 0; q < kCombineQ; ++q) {
    w[q] = blk * kCombineWin + ((int64_t)q * 256 + threadIdx.x) * 4;
#pragma unroll
    for (int a = 0; a < NACC; ++a) m[q][a] = make_uint4(0u, 0u, 0u, 0u);
  }
  for (int g0 = 0; g0 < p.ngroups; g0 += GB) {
    u32x2_v h[GB][kCombineQ][NACC];
#pragma unroll
    for (int u = 0; u < GB; ++u)
#pragma unroll
      for (int q = 0; q < kCombineQ; ++q)
#pragma unroll
        for (int a = 0; a < NACC; ++a) {
          const int64_t o = ((int64_t)(g0 + u) * NACC + a) * p.pstride + w[q];
          h[u][q][a] = (g0 + u < p.ngroups && w[q] < p.nwin)
                           ? *(const __attribute__((address_space(1))) u32x2_v*)gbl(p.part + o)
                           : u32x2_v{0u, 0u};
        }
#pragma unroll
    for (int u = 0; u < GB; ++u)
#pragma unroll
      for (int q = 0; q < kCombineQ; ++q)
#pragma unroll
        for (int a = 0; a < NACC; ++a) {
          const u32x2_v v = h[u][q][a];
          m[q][a] = make_uint4(m[q][a].x + (v[0] & 0xFFFFu), m[q][a].y + (v[0] >> 16),
                               m[q][a].z + (v[1] & 0xFFFFu), m[q][a].w + (v[1] >> 16));
        }
  }
#pragma unroll
  for (int q = 0; q < kCombineQ; ++q) {
    if (w[q] >= p.nwin) continue;
    // the L1 terms, exact in integers
    float sc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float s = 0.f;
#pragma unroll
      for (int a = 0; a < NACC; ++a) {
        const uint32_t mi = i == 0 ? m[q][a].x : i == 1 ? m[q][a].y : i == 2 ? m[q][a].z : m[q][a].w;
        s = fmaf(p.wt[a], (float)(p.area2[a] + p.cmul[a] * (int)mi), s);
      }
      sc[i] = -s;
    }
    const int nv = (int)min((int64_t)4, p.nwin - w[q]);
    if (nv == 4 && p.vec_out) {
      *(__attribute__((address_space(1))) f32x4_v*)gbl(p.heatmap + w[q]) = f32x4_v{sc[0], sc[1], sc[2], sc[3]};
    } else {
      for (int i = 0; i < nv; ++i) gbl(p.heatmap)[w[q] + i] = sc[i];
    }
    for (int i = 0; i < nv; ++i) {
      const unsigned long long k2 = best_key(sc[i], (uint32_t)(w[q] + i));
      key = k2 > key ? k2 : key;
    }
  }
  block_max_to(key, p.best);
}

template <int NACC>
__global__ __launch_bounds__(256) void score_combine_kernel(CombineParams p) {
  combine_body<NACC>(p, blockIdx.x);
}

template <int NACC>
__global__ __launch_bounds__(256) void score_combine_batch_kernel(const CombineParams* __restrict__ tab,
                                                                  const uint32_t* __restrict__ blk) {
  const CombineParams& p = tab[blk[blockIdx.x]];
  combine_body<NACC>(p, (int64_t)(blockIdx.x - p.b0));
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

// Geometry of the on-chip score for one template: tile width, the stored
// sums (full window, then bins merged by weight) and their weights / areas.
struct TilePlan {
  bool ok;
  bool uni;           // every bin has one weight: two sums
  int kg;             // channels per block (16 or 32)
  bool sad;           // blocks sum |T_j - C_j| (every stored sum < 2^16)
  int txw;
  int nacc;
  uint32_t cmask[kMaxCls];
  float wt[kMaxAcc];
  int area2[kMaxAcc];
};

// Tiles are as wide as the LDS rows allow (at most kTXW windows, at least 32).
// wide: 32-channel blocks where the grid allows them (G <= 3; they hold 4 G
// rows of LDS histograms and prefixes, 142 KB at G = 3).
TilePlan plan_tile(const DeviceTemplate& t, bool wide = false) {
  TilePlan pl{};
  if (!t.grid.valid) return pl;
  const int G = t.grid.g;
  const int NF = 1 + G * G;
  if (G < 1 || G > 4 || t.geom.kpad % 16 || t.n_filters != NF) return pl;
  pl.kg = (wide && G <= 3 && t.geom.kpad % 32 == 0) ? 32 : 16;
  int maxband = 0;
  for (int b = 0; b < G; ++b) maxband = std::max(maxband, t.grid.ye[b + 1] - t.grid.ye[b]);
  pl.txw = std::min(kTXW, kColsMax + 1 - t.w);
  if (pl.txw < 32) return pl;
  if ((int64_t)maxband * (kColsMax + 1) >= 65536) return pl;   // u16 prefix counts
  // bins of equal weight share a sum: classes in order of first appearance
  std::vector<float> wd;
  int cls[17] = {};
  for (int f = 1; f < NF; ++f) {
    const auto it = std::find(wd.begin(), wd.end(), t.weights[f]);
    cls[f] = (int)(it - wd.begin());
    if (it == wd.end()) wd.push_back(t.weights[f]);
  }
  // more distinct bin weights than stored sums: the integral-image path
  if ((int)wd.size() > kMaxCls) return pl;
  pl.uni = wd.size() == 1;
  pl.nacc = 1 + (int)wd.size();
  for (int f = 0; f < NF; ++f) {
    const int32_t* b = &t.boxes[(size_t)f * 4];
    const int area = (b[2] - b[0]) * (b[3] - b[1]);
    const int a = f == 0 ? 0 : 1 + cls[f];
    pl.wt[a] = t.weights[f];
    pl.area2[a] += 2 * area;
    if (f > 0) pl.cmask[cls[f]] |= 1u << f;
  }
  if ((int64_t)t.w * t.h > 65535) return pl;   // 16-bit partial sums
  // a group's sum of |T_j - C_j| over a stored sum's filters is at most
  // twice their area: 16 bits hold it unless the template is large
  pl.sad = true;
  for (int a = 0; a < pl.nacc; ++a) pl.sad = pl.sad && pl.area2[a] <= 65535;
  pl.ok = true;
  return pl;
}

// The default block width of a single pair: 32-channel blocks where the grid
// allows them (on 1024 x 1024 maps they scored 2 x 2 and 3 x 3 grids 2-20%
// faster than 16-channel blocks); batches default to 16-channel blocks.
bool default_wide(const DeviceTemplate& t) { return t.grid.valid && t.grid.g <= 3; }

// Kernel arguments of one pair's tile and combine kernels.
struct PairTables {
  TileParams tp;
  CombineParams cp;
  int G;
  bool uni;
  int kg;
  bool sad;
  int ny;
  int64_t ncblk;   // combine blocks (0: the tile kernel forms the scores)
};

void make_pair(const DeviceTemplate& t, const TilePlan& pl, const uint8_t* labels, int H, int W, int tyw,
               uint16_t* part, float* heatmap, unsigned long long* best, PairTables* o) {
  const int ow = W - t.w + 1, oh = H - t.h + 1;
  // equal tile widths
  const int nx = (ow + pl.txw - 1) / pl.txw;
  TileParams& tp = o->tp;
  tp = TileParams{};
  tp.labels = labels;
  tp.H = H;
  tp.W = W;
  tp.w = t.w;
  tp.h = t.h;
  tp.ow = ow;
  tp.oh = oh;
  tp.txw = (ow + nx - 1) / nx;
  tp.tyw = std::max(1, std::min(tyw, oh));
  tp.kpad = t.geom.kpad;
  const int G = t.grid.g;
  for (int i = 0; i <= G; ++i) {
    tp.xe[i] = t.grid.xe[i];
    tp.ye[i] = t.grid.ye[i];
  }
  tp.t16 = t.d_counts16;
  tp.pstride = ((int64_t)ow * oh + 3) / 4 * 4;
  tp.nacc = pl.nacc;
  for (int c = 0; c < kMaxCls; ++c) tp.cmask[c] = pl.cmask[c];
  tp.nx = nx;
  tp.ng = t.geom.kpad / pl.kg;
  for (int a = 0; a < kMaxAcc; ++a) {
    tp.wt[a] = pl.wt[a];
    tp.area2[a] = pl.sad ? 0 : pl.area2[a];
    tp.cmul[a] = pl.sad ? 1 : -2;
  }
  tp.heatmap = heatmap;
  tp.best = best;
  tp.part = tp.ng > 1 ? part : nullptr;
  o->G = G;
  o->uni = pl.uni;
  o->kg = pl.kg;
  o->sad = pl.sad;
  o->ny = (oh + tp.tyw - 1) / tp.tyw;
  CombineParams& cp = o->cp;
  cp = CombineParams{};
  cp.part = tp.part;
  cp.nwin = (int64_t)ow * oh;
  cp.pstride = tp.pstride;
  cp.vec_out = ((uintptr_t)heatmap % 16) == 0;
  cp.ngroups = tp.ng;
  for (int a = 0; a < kMaxAcc; ++a) {
    cp.wt[a] = pl.wt[a];
    cp.area2[a] = pl.sad ? 0 : pl.area2[a];
    cp.cmul[a] = pl.sad ? 1 : -2;
  }
  cp.heatmap = heatmap;
  cp.best = best;
  o->ncblk = tp.ng > 1 ? (cp.nwin + kCombineWin - 1) / kCombineWin : 0;
}

size_t partial_bytes(const DeviceTemplate& t, const TilePlan& pl, int H, int W) {
  const int ng = t.geom.kpad / pl.kg;
  if (ng <= 1) return 0;
  const int64_t nwin = (int64_t)(H - t.h + 1) * (W - t.w + 1);
  return (size_t)ng * pl.nacc * ((nwin + 3) / 4 * 4) * 2;
}

template <int G, bool UNI, int KG, bool SAD>
hipError_t go_tile(const TileParams& tp, int ny, hipStream_t s) {
  const dim3 grid((unsigned)tp.nx, (unsigned)ny, (unsigned)tp.ng);
  hipLaunchKernelGGL((score_tile_kernel<G, UNI, KG, SAD>), grid, dim3(kTXW * (KG / 8)), 0, s, tp);
  return hipGetLastError();
}

template <int G, bool UNI, int KG, bool SAD>
hipError_t go_tile_b(const TileParams* tab, const uint32_t* blk, uint32_t nblk, hipStream_t s) {
  hipLaunchKernelGGL((score_tile_batch_kernel<G, UNI, KG, SAD>), dim3(nblk), dim3(kTXW * (KG / 8)), 0, s, tab,
                     blk);
  return hipGetLastError();
}

template <bool SAD>
hipError_t go_tile_sad(int G, bool uni, int kg, const TileParams& tp, int ny, const TileParams* tab,
                       const uint32_t* blk, uint32_t nblk, hipStream_t s) {
#define VQ_TILE(g, u, k) \
  return tab ? go_tile_b<g, u, k, SAD>(tab, blk, nblk, s) : go_tile<g, u, k, SAD>(tp, ny, s)
  if (kg == 32) {
    switch (G * 2 + (uni ? 1 : 0)) {
      case 2: VQ_TILE(1, false, 32);
      case 3: VQ_TILE(1, true, 32);
      case 4: VQ_TILE(2, false, 32);
      case 5: VQ_TILE(2, true, 32);
      case 6: VQ_TILE(3, false, 32);
      case 7: VQ_TILE(3, true, 32);
      default: return hipErrorInvalidValue;
    }
  }
  if (kg != 16) return hipErrorInvalidValue;
  switch (G * 2 + (uni ? 1 : 0)) {
    case 2: VQ_TILE(1, false, 16);
    case 3: VQ_TILE(1, true, 16);
    case 4: VQ_TILE(2, false, 16);
    case 5: VQ_TILE(2, true, 16);
    case 6: VQ_TILE(3, false, 16);
    case 7: VQ_TILE(3, true, 16);
    case 8: VQ_TILE(4, false, 16);
    case 9: VQ_TILE(4, true, 16);
    default: return hipErrorInvalidValue;
  }
#undef VQ_TILE
}

// One pair (tab == nullptr) or a batch.  32-channel blocks for G <= 3 only.
hipError_t go_tile_any(int G, bool uni, int kg, bool sad, const TileParams& tp, int ny, const TileParams* tab,
                       const uint32_t* blk, uint32_t nblk, hipStream_t s) {
  return sad ? go_tile_sad<true>(G, uni, kg, tp, ny, tab, blk, nblk, s)
             : go_tile_sad<false>(G, uni, kg, tp, ny, tab, blk, nblk, s);
}

// Static LDS of a tile block: histograms and prefixes of G * KG / 8 rows,
// plus every pair group's sums of a row.
size_t tile_lds_bytes(int G, bool uni, int kg) {
  const int pq = kg / 8;
  return (size_t)2 * G * pq * kHS * 16 + (size_t)pq * (uni ? 2 : kMaxAcc) * kTXW * 2;
}

// Tile blocks resident per compute unit (160 KB of LDS, 2048 threads).
int tile_blocks_per_cu(int G, bool uni, int kg) {
  const int by_threads = 2048 / (kTXW * (kg / 8));
  const int by_lds = (int)(163840 / std::max<size_t>(tile_lds_bytes(G, uni, kg), 1));
  return std::max(1, std::min(by_threads, by_lds));
}

template <int NACC>
hipError_t go_comb(const CombineParams& cp, int64_t nblk, const CombineParams* tab, const uint32_t* blk,
                   hipStream_t s) {
  if (tab)
    hipLaunchKernelGGL((score_combine_batch_kernel<NACC>), dim3((unsigned)nblk), dim3(256), 0, s, tab, blk);
  else
    hipLaunchKernelGGL((score_combine_kernel<NACC>), dim3((unsigned)nblk), dim3(256), 0, s, cp);
  return hipGetLastError();
}

hipError_t go_combine_any(int nacc, const CombineParams& cp, int64_t nblk, const CombineParams* tab,
                          const uint32_t* blk, hipStream_t s) {
#define VQ_COMB(n) return go_comb<n>(cp, nblk, tab, blk, s)
  switch (nacc) {
    case 2: VQ_COMB(2);
    case 3: VQ_COMB(3);
    case 4: VQ_COMB(4);
    case 5: VQ_COMB(5);
    default: return hipErrorInvalidValue;
  }
#undef VQ_COMB
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

size_t fused_partial_bytes(const DeviceTemplate& t, int H, int W) {
  TilePlan pl = plan_tile(t);
  if (!pl.ok) return 0;
  return partial_bytes(t, pl, H, W);
}

hipError_t launch_score_fused(const ScoreArgs& a, hipStream_t s, size_t* lds_bytes_out) {
  const DeviceTemplate& t = *a.t;
  const bool wide = a.kgsel == 0 ? default_wide(t) : a.kgsel == 2;
  TilePlan pl = plan_tile(t, wide);
  if (!pl.ok) return hipErrorInvalidConfiguration;
  if (partial_bytes(t, pl, a.H, a.W) > 0 && !a.partials) return hipErrorInvalidValue;
  // tile height from the caller (autotuned) or the default
  const int tyw = a.tyw > 0 ? a.tyw : fused_default_tyw(t, a.H, a.W, a.n_cu, wide);
  PairTables pt;
  make_pair(t, pl, a.labels, a.H, a.W, tyw, (uint16_t*)a.partials, a.heatmap, a.best, &pt);
  if (lds_bytes_out) *lds_bytes_out = tile_lds_bytes(pt.G, pt.uni, pt.kg);
  timing_begin(K_SCORE_FUSED);
  hipError_t e = go_tile_any(pt.G, pt.uni, pt.kg, pt.sad, pt.tp, pt.ny, nullptr, nullptr, 0, s);
  timing_end(K_SCORE_FUSED);
  if (e != hipSuccess || pt.ncblk == 0) return e;
  timing_begin(K_SCORE_COMBINE);
  e = go_combine_any(pl.nacc, pt.cp, pt.ncblk, nullptr, nullptr, s);
  timing_end(K_SCORE_COMBINE);
  return e;
}

bool plan_score_batch(const std::vector<ScoreBatchItem>& items, void* part, ScoreBatchPlan* out, bool wide) {
  out->blob.clear();
  out->launches.clear();
  out->part_bytes = 0;
  std::vector<PairTables> pts(items.size());
  std::vector<TilePlan> pls(items.size());
  for (size_t i = 0; i < items.size(); ++i) {
    const ScoreBatchItem& it = items[i];
    pls[i] = plan_tile(*it.t, wide);
    if (!pls[i].ok || it.tyw < 1) return false;
    const size_t pb = partial_bytes(*it.t, pls[i], it.H, it.W);
    uint16_t* pp = part ? (uint16_t*)((char*)part + out->part_bytes) : nullptr;
    make_pair(*it.t, pls[i], it.labels, it.H, it.W, it.tyw, pp, it.heatmap, it.best, &pts[i]);
    out->part_bytes += align_up(pb, 256);
  }
  // tile launches per (G, uniform bins, channels per block); pairs with the
  // largest templates (the costliest tile set-up) first
  std::vector<size_t> order(items.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
    return (int64_t)items[a].t->w * items[a].t->h > (int64_t)items[b].t->w * items[b].t->h;
  });
  auto put = [&](const void* src, size_t bytes) {
    const size_t off = align_up(out->blob.size(), 64);
    out->blob.resize(off + bytes);
    std::memcpy(out->blob.data() + off, src, bytes);
    return off;
  };
  for (int kg : {32, 16})
  for (int G = 1; G <= 4; ++G)
  for (int sad = 1; sad >= 0; --sad)
    for (int u = 0; u < 2; ++u) {
      std::vector<TileParams> tab;
      std::vector<uint32_t> blk;
      for (size_t i : order) {
        PairTables& pt = pts[i];
        if (pt.G != G || pt.uni != (u == 1) || pt.kg != kg || pt.sad != (sad == 1)) continue;
        pt.tp.b0 = (uint32_t)blk.size();
        const int64_t nb = (int64_t)pt.tp.nx * pt.ny * pt.tp.ng;
        if ((int64_t)blk.size() + nb > 0x7FFFFFFF) return false;
        blk.insert(blk.end(), (size_t)nb, (uint32_t)tab.size());
        tab.push_back(pt.tp);
      }
      if (tab.empty()) continue;
      ScoreBatchLaunch l{};
      l.kind = 0;
      l.G = G;
      l.uni = u;
      l.kg = kg;
      l.sad = sad;
      l.tab_off = put(tab.data(), tab.size() * sizeof(TileParams));
      l.blk_off = put(blk.data(), blk.size() * 4);
      l.nblk = (uint32_t)blk.size();
      out->launches.push_back(l);
    }
  for (int nacc : {2, 3, 4, 5}) {
      std::vector<CombineParams> tab;
      std::vector<uint32_t> blk;
      for (size_t i : order) {
        PairTables& pt = pts[i];
        if (pt.ncblk == 0 || pls[i].nacc != nacc) continue;
        pt.cp.b0 = (uint32_t)blk.size();
        if ((int64_t)blk.size() + pt.ncblk > 0x7FFFFFFF) return false;
        blk.insert(blk.end(), (size_t)pt.ncblk, (uint32_t)tab.size());
        tab.push_back(pt.cp);
      }
      if (tab.empty()) continue;
      ScoreBatchLaunch l{};
      l.kind = 1;
      l.nacc = nacc;
      l.tab_off = put(tab.data(), tab.size() * sizeof(CombineParams));
      l.blk_off = put(blk.data(), blk.size() * 4);
      l.nblk = (uint32_t)blk.size();
      out->launches.push_back(l);
    }
  return true;
}

hipError_t launch_score_batch(const ScoreBatchPlan& pl, const uint8_t* d_blob, hipStream_t s) {
  for (const ScoreBatchLaunch& l : pl.launches) {
    const uint32_t* blk = (const uint32_t*)(d_blob + l.blk_off);
    hipError_t e;
    if (l.kind == 0) {
      timing_begin(K_SCORE_FUSED);
      e = go_tile_any(l.G, l.uni != 0, l.kg, l.sad != 0, TileParams{}, 0,
                      (const TileParams*)(d_blob + l.tab_off), blk, l.nblk, s);
      timing_end(K_SCORE_FUSED);
    } else {
      timing_begin(K_SCORE_COMBINE);
      e = go_combine_any(l.nacc, CombineParams{}, l.nblk, (const CombineParams*)(d_blob + l.tab_off),
                         blk, s);
      timing_end(K_SCORE_COMBINE);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

bool fused_supported(const DeviceTemplate& t) { return plan_tile(t).ok; }

bool fused_wide_allowed(const DeviceTemplate& t) { return plan_tile(t, true).kg == 32; }

bool fused_default_wide(const DeviceTemplate& t) { return default_wide(t); }

int fused_groups(const DeviceTemplate& t) {
  const TilePlan pl = plan_tile(t);
  return pl.ok ? t.geom.kpad / pl.kg : t.geom.kpad / 16;
}

// Tiles fill whole rounds of the blocks resident per compute unit (at least
// 8 rows).
int fused_default_tyw(const DeviceTemplate& t, int H, int W, int n_cu, bool wide) {
  TilePlan pl = plan_tile(t, wide);
  if (!pl.ok) return 8;
  const int ow = W - t.w + 1, oh = H - t.h + 1;
  const int nx = (ow + pl.txw - 1) / std::max(pl.txw, 1);
  const int per_row = nx * (t.geom.kpad / pl.kg);
  const int slots = tile_blocks_per_cu(t.grid.g, pl.uni, pl.kg) * std::max(n_cu, 1);
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
