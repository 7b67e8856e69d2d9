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
  int kpad, kg;       // channels (padded) and channels per block (group)
  int qs, hs;         // LDS row strides (dwords) of Q and H
  int xe[5], ye[5];
  const uint32_t* t16;  // [nf][kpad/2] template counts, u16 pairs
  uint16_t* part;       // [n_groups][nf][oh*ow] sum_j min(T_j, C_j) per group
};

constexpr int kTYW = 32;    // window rows per tile
constexpr int kFT = 1024;   // threads per block
constexpr int kSEG = 8;     // columns per prefix segment

// Inclusive prefix sum across the 64 lanes of a wave with DPP: row_shr 1, 2,
// 4, 8 inside each row of 16 lanes, then row_bcast 15 and 31 carry the row
// totals into the following rows.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);
  return x;
}

// Block (x tile of TXW windows, y tile of kTYW rows, channel group of KG
// channels).  NP = kFT / TXW threads per window, each taking every NP-th
// channel pair of the group.
//
// LDS per band b and channel quad q: Q[b][q][c] (four uint8 column counts),
// the segment totals T[b][q][s] = sum of Q over the kSEG columns of segment s
// (two packed u16 pairs), kept up to date by the vertical updates, and the
// prefix H[b][pair][c].  Per window row: vertical update (Q and T) | scan of T
// per (b, q) row -> segment offsets | write H = offset + running sum inside
// the segment | evaluate windows.
template <int G, int TXW, int KG>
__global__ __launch_bounds__(kFT) void score_partial_kernel(FusedParams p) {
  constexpr int NF = 1 + G * G;
  constexpr int NP = kFT / TXW;
  constexpr int KQ = KG / 4, KP = KG / 2;
  extern __shared__ uint32_t sm[];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int x0 = blockIdx.x * TXW, y0 = blockIdx.y * kTYW;
  const int grp = blockIdx.z;
  const int j0 = grp * KG;                            // first channel of the group
  const int txv = min(TXW, p.ow - x0), tyv = min(kTYW, p.oh - y0);
  const int cols = txv + p.w - 1;
  const int nseg = (cols + kSEG - 1) / kSEG;          // <= 64
  uint32_t* Q = sm;                                   // [G][KQ][qs]
  uint32_t* Hs = Q + G * KQ * p.qs;                   // [G][KP][hs]
  uint32_t* segt = Hs + G * KP * p.hs;                // [G][KQ][64][2] totals
  uint32_t* sego = segt + G * KQ * 64 * 2;            // [G][KQ][64][2] offsets
  uint32_t* red = sego + G * KQ * 64 * 2;             // [NF][TXW]

  for (int i = tid; i < G * KQ * p.qs; i += kFT) Q[i] = 0u;
  for (int i = tid; i < NF * TXW; i += kFT) red[i] = 0u;
  __syncthreads();
  // initial band histograms of the group's channels: items of 8 rows of one
  // column, the 8 label loads issued together
  const int nrc = (p.h + 7) / 8;
  for (int i = tid; i < nrc * cols; i += kFT) {
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
      if ((unsigned)l8[r] < (unsigned)KG)
        atomicAdd(&Q[(b * KQ + (l8[r] >> 2)) * p.qs + c], 1u << (8 * (l8[r] & 3)));
    }
  }
  __syncthreads();
  // initial segment totals
  for (int it = tid; it < G * KQ * 64; it += kFT) {
    const int bq = it % (G * KQ), seg = it / (G * KQ);
    uint32_t r0 = 0u, r1 = 0u;
    if (seg < nseg) {
      const uint32_t* qrow = Q + bq * p.qs + seg * kSEG;
#pragma unroll
      for (int i = 0; i < kSEG; ++i) {
        const uint32_t v = (seg * kSEG + i < cols) ? qrow[i] : 0u;
        r0 += (v & 0xFFu) | ((v & 0xFF00u) << 8);
        r1 += ((v >> 16) & 0xFFu) | ((v >> 8) & 0xFF0000u);
      }
    }
    segt[(bq * 64 + seg) * 2] = r0;
    segt[(bq * 64 + seg) * 2 + 1] = r1;
  }

  const int xl = tid % TXW;
  const int part = __builtin_amdgcn_readfirstlane(tid / TXW);   // uniform per wave
  const int64_t nwin = (int64_t)p.ow * p.oh;
  // template counts of this thread's channel pairs, in registers
  constexpr int PPT = (KP + NP - 1) / NP;             // pairs per thread
  uint32_t tcr[PPT][NF];
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int pl = part + NP * i;
#pragma unroll
    for (int f = 0; f < NF; ++f)
      tcr[i][f] = (pl < KP) ? p.t16[f * (p.kpad / 2) + j0 / 2 + pl] : 0u;
  }
  // labels entering / leaving each band at the next row step, prefetched
  int lo[G], li[G];
  auto fetch = [&](int ynext, int c) {
#pragma unroll
    for (int b = 0; b < G; ++b) {
      lo[b] = (int)p.labels[(int64_t)(ynext - 1 + p.ye[b]) * p.W + x0 + c] - j0;
      li[b] = (int)p.labels[(int64_t)(ynext - 1 + p.ye[b + 1]) * p.W + x0 + c] - j0;
    }
  };
  // columns are owned by threads tid < cols (cols <= TXW + 254 < kFT)
  if (tyv > 1 && tid < cols) fetch(y0 + 1, tid);

  for (int dy = 0; dy < tyv; ++dy) {
    const int y = y0 + dy;
    if (dy > 0 && tid < cols) {
      const int c = tid, sg = c / kSEG;
#pragma unroll
      for (int b = 0; b < G; ++b) {
        if (lo[b] == li[b]) continue;
        if ((unsigned)lo[b] < (unsigned)KG) {
          const int q = lo[b] >> 2;
          Q[(b * KQ + q) * p.qs + c] -= 1u << (8 * (lo[b] & 3));
          atomicSub(&segt[((b * KQ + q) * 64 + sg) * 2 + ((lo[b] >> 1) & 1)], 1u << (16 * (lo[b] & 1)));
        }
        if ((unsigned)li[b] < (unsigned)KG) {
          const int q = li[b] >> 2;
          Q[(b * KQ + q) * p.qs + c] += 1u << (8 * (li[b] & 3));
          atomicAdd(&segt[((b * KQ + q) * 64 + sg) * 2 + ((li[b] >> 1) & 1)], 1u << (16 * (li[b] & 1)));
        }
      }
    }
    __syncthreads();
    // ---- per (band, quad) row, one wave: exclusive scan of the segment
    // totals -> offsets; entry `cols` of H receives the row total
    for (int bq = wv; bq < G * KQ; bq += kFT / 64) {
      const int b = bq / KQ, qq = bq % KQ;
      const uint32_t t0 = lane < nseg ? segt[(bq * 64 + lane) * 2] : 0u;
      const uint32_t t1 = lane < nseg ? segt[(bq * 64 + lane) * 2 + 1] : 0u;
      const uint32_t i0 = wave_incl_scan(t0), i1 = wave_incl_scan(t1);
      sego[(bq * 64 + lane) * 2] = i0 - t0;
      sego[(bq * 64 + lane) * 2 + 1] = i1 - t1;
      if (lane == nseg - 1) {
        uint32_t* h0 = Hs + (b * KP + 2 * qq) * p.hs;
        h0[cols] = i0;
        h0[p.hs + cols] = i1;
      }
    }
    __syncthreads();
    // ---- H = segment offset + running sum inside the segment; consecutive
    // lanes take different rows (odd row stride: no bank conflicts)
    for (int it = tid; it < G * KQ * nseg; it += kFT) {
      const int bq = it % (G * KQ), seg = it / (G * KQ);
      const int b = bq / KQ, qq = bq % KQ;
      const int c0 = seg * kSEG;
      const uint32_t* qrow = Q + bq * p.qs + c0;
      uint32_t* h0 = Hs + (b * KP + 2 * qq) * p.hs + c0;
      uint32_t* h1 = h0 + p.hs;
      uint32_t v[kSEG];
#pragma unroll
      for (int i = 0; i < kSEG; ++i) v[i] = (c0 + i < cols) ? qrow[i] : 0u;
      uint32_t r0 = sego[(bq * 64 + seg) * 2], r1 = sego[(bq * 64 + seg) * 2 + 1];
#pragma unroll
      for (int i = 0; i < kSEG; ++i) {
        h0[i] = r0;
        h1[i] = r1;
        r0 += (v[i] & 0xFFu) | ((v[i] & 0xFF00u) << 8);
        r1 += ((v[i] >> 16) & 0xFFu) | ((v[i] >> 8) & 0xFF0000u);
      }
    }
    __syncthreads();
    // next row's labels are requested now and consumed after the evaluation
    if (dy + 1 < tyv && tid < cols) fetch(y + 1, tid);
    // ---- evaluate windows: thread (xl, part) takes every NP-th pair
    uint32_t acc[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] = 0u;
    if (xl < txv) {
#pragma unroll
      for (int i = 0; i < PPT; ++i) {
        const int pl = part + NP * i;
        if (pl >= KP) break;
        uint32_t full = 0u;
#pragma unroll
        for (int b = 0; b < G; ++b) {
          const uint32_t* hrow = Hs + (b * KP + pl) * p.hs + xl;
          uint32_t hb[G + 1];
#pragma unroll
          for (int a = 0; a <= G; ++a) hb[a] = hrow[p.xe[a]];
#pragma unroll
          for (int a = 0; a < G; ++a)
            acc[1 + b * G + a] = pk_min_add(acc[1 + b * G + a], hb[a + 1] - hb[a], tcr[i][1 + b * G + a]);
          full += hb[G] - hb[0];
        }
        acc[0] = pk_min_add(acc[0], full, tcr[i][0]);
      }
    }
    // ---- combine the NP parts and write the group's partial sums
    if (part > 0 && xl < txv) {
#pragma unroll
      for (int f = 0; f < NF; ++f) atomicAdd(&red[f * TXW + xl], acc[f]);
    }
    __syncthreads();
    if (part == 0 && xl < txv) {
      const int64_t win = (int64_t)y * p.ow + x0 + xl;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const uint32_t t = acc[f] + red[f * TXW + xl];
        red[f * TXW + xl] = 0u;
        p.part[((int64_t)grp * NF + f) * nwin + win] = (uint16_t)((t & 0xFFFFu) + (t >> 16));
      }
    }
  }
}

// Sums the groups' partials, forms eq. 2 and the argmax.
struct CombineParams {
  const uint16_t* part;
  int64_t nwin;
  int ow, ngroups, nf;
  float wt[17];
  int area[17];
  float* heatmap;
  unsigned long long* best;
};

// Eight windows per thread, 16-byte loads of the partial sums; the group
// loop is unrolled so every load of a filter is in flight at once.
template <int NF, int NG>
__global__ __launch_bounds__(256) void score_combine_kernel(CombineParams p) {
  const int64_t w0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 8;
  unsigned long long key = 0ull;
  if (w0 < p.nwin) {
    const int nv = (int)min((int64_t)8, p.nwin - w0);
    const bool vec = (nv == 8) && ((p.nwin & 7) == 0);
    float s[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) s[i] = 0.f;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      int mins[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) mins[i] = 0;
      if (vec) {
        uint4 v[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) v[g] = *(const uint4*)(p.part + ((int64_t)g * NF + f) * p.nwin + w0);
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          const uint32_t ws[4] = {v[g].x, v[g].y, v[g].z, v[g].w};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            mins[2 * i] += (int)(ws[i] & 0xFFFFu);
            mins[2 * i + 1] += (int)(ws[i] >> 16);
          }
        }
      } else {
        for (int g = 0; g < NG; ++g)
          for (int i = 0; i < nv; ++i) mins[i] += p.part[((int64_t)g * NF + f) * p.nwin + w0 + i];
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) s[i] = fmaf(p.wt[f], (float)(2 * p.area[f] - 2 * mins[i]), s[i]);
    }
    for (int i = 0; i < nv; ++i) {
      const float score = -s[i];
      p.heatmap[w0 + i] = score;
      const unsigned long long k2 = best_key(score, (uint32_t)(w0 + i));
      key = k2 > key ? k2 : key;
    }
  }
  key = wave_max_u64(key);
  if ((threadIdx.x & 63) == 0 && key) atomicMax(p.best, key);
}

template <int NF>
hipError_t go_combine_nf(const CombineParams& cp, hipStream_t s) {
  const dim3 grid((unsigned)((cp.nwin + 2047) / 2048)), blk(256);
  switch (cp.ngroups) {
    case 1: hipLaunchKernelGGL((score_combine_kernel<NF, 1>), grid, blk, 0, s, cp); break;
    case 2: hipLaunchKernelGGL((score_combine_kernel<NF, 2>), grid, blk, 0, s, cp); break;
    case 4: hipLaunchKernelGGL((score_combine_kernel<NF, 4>), grid, blk, 0, s, cp); break;
    case 8: hipLaunchKernelGGL((score_combine_kernel<NF, 8>), grid, blk, 0, s, cp); break;
    case 16: hipLaunchKernelGGL((score_combine_kernel<NF, 16>), grid, blk, 0, s, cp); break;
    case 32: hipLaunchKernelGGL((score_combine_kernel<NF, 32>), grid, blk, 0, s, cp); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t go_combine(const CombineParams& cp, hipStream_t s) {
  switch (cp.nf) {
    case 2: return go_combine_nf<2>(cp, s);
    case 5: return go_combine_nf<5>(cp, s);
    case 10: return go_combine_nf<10>(cp, s);
    case 17: return go_combine_nf<17>(cp, s);
    default: return hipErrorInvalidValue;
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
  int txw, kg, qs, hs;
  size_t lds;
};

FusedPlan plan_fused(const DeviceTemplate& t) {
  FusedPlan pl{};
  const int G = t.grid.g;
  int maxband = 0;
  for (int b = 0; b < G; ++b) maxband = std::max(maxband, t.grid.ye[b + 1] - t.grid.ye[b]);
  const int kpad = t.geom.kpad;
  const int NF = 1 + G * G;
  for (int txw = 256; txw >= 64; txw /= 2) {
    const int colsmax = txw + t.w - 1;
    if ((int64_t)maxband * colsmax >= 65536) continue;   // 16-bit prefix would overflow
    if ((colsmax + kSEG - 1) / kSEG > 64) continue;       // segment totals scanned by one wave
    // padded so the unrolled segment loads and stores stay in their rows
    const int qs = ((colsmax + kSEG - 1) / kSEG * kSEG) | 1;
    const int hs = ((colsmax + kSEG) / kSEG * kSEG + 1) | 1;
    // 16 channels per block keeps LDS under 80 KB: two blocks per CU
    for (int kg = 16; kg >= 8; kg /= 2) {
      if (kpad % kg) continue;
      size_t lds = 4 * ((size_t)G * (kg / 4) * qs + (size_t)G * (kg / 2) * hs +
                        2 * (size_t)G * (kg / 4) * 64 * 2 + (size_t)NF * txw);
      if (lds <= 160 * 1024) {
        pl.ok = true;
        pl.txw = txw;
        pl.kg = kg;
        pl.qs = qs;
        pl.hs = hs;
        pl.lds = lds;
        return pl;
      }
    }
  }
  return pl;
}

template <int G, int TXW, int KG>
hipError_t go_fused(const FusedParams& fp, const FusedPlan& pl, hipStream_t s) {
  auto kern = score_partial_kernel<G, TXW, KG>;
  if (pl.lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.lds);
    if (e != hipSuccess) return e;
  }
  dim3 grid((fp.ow + TXW - 1) / TXW, (fp.oh + kTYW - 1) / kTYW, fp.kpad / KG);
  hipLaunchKernelGGL(kern, grid, dim3(kFT), pl.lds, s, fp);
  return hipGetLastError();
}

template <int G, int TXW>
hipError_t go_fused_k(const FusedParams& fp, const FusedPlan& pl, hipStream_t s) {
  return pl.kg == 16 ? go_fused<G, TXW, 16>(fp, pl, s) : go_fused<G, TXW, 8>(fp, pl, s);
}

}  // namespace

size_t fused_partial_bytes(const DeviceTemplate& t, int H, int W) {
  FusedPlan pl = plan_fused(t);
  if (!pl.ok) return 0;
  const int64_t nwin = (int64_t)(H - t.h + 1) * (W - t.w + 1);
  return (size_t)(t.geom.kpad / pl.kg) * t.n_filters * nwin * 2;
}

hipError_t launch_score_fused(const ScoreArgs& a, hipStream_t s, size_t* lds_bytes_out) {
  const DeviceTemplate& t = *a.t;
  if (!t.grid.valid || !a.partials) return hipErrorInvalidValue;
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
  fp.kg = pl.kg;
  fp.qs = pl.qs;
  fp.hs = pl.hs;
  const int G = t.grid.g;
  for (int i = 0; i <= G; ++i) {
    fp.xe[i] = t.grid.xe[i];
    fp.ye[i] = t.grid.ye[i];
  }
  fp.t16 = t.d_counts16;
  fp.part = (uint16_t*)a.partials;
  if (lds_bytes_out) *lds_bytes_out = pl.lds;
  timing_begin(K_SCORE_FUSED);
  hipError_t e;
  switch (pl.txw * 8 + G) {
    case 256 * 8 + 1: e = go_fused_k<1, 256>(fp, pl, s); break;
    case 256 * 8 + 2: e = go_fused_k<2, 256>(fp, pl, s); break;
    case 256 * 8 + 3: e = go_fused_k<3, 256>(fp, pl, s); break;
    case 256 * 8 + 4: e = go_fused_k<4, 256>(fp, pl, s); break;
    case 128 * 8 + 1: e = go_fused_k<1, 128>(fp, pl, s); break;
    case 128 * 8 + 2: e = go_fused_k<2, 128>(fp, pl, s); break;
    case 128 * 8 + 3: e = go_fused_k<3, 128>(fp, pl, s); break;
    case 128 * 8 + 4: e = go_fused_k<4, 128>(fp, pl, s); break;
    case 64 * 8 + 1: e = go_fused_k<1, 64>(fp, pl, s); break;
    case 64 * 8 + 2: e = go_fused_k<2, 64>(fp, pl, s); break;
    case 64 * 8 + 3: e = go_fused_k<3, 64>(fp, pl, s); break;
    case 64 * 8 + 4: e = go_fused_k<4, 64>(fp, pl, s); break;
    default: e = hipErrorInvalidValue;
  }
  timing_end(K_SCORE_FUSED);
  if (e != hipSuccess) return e;
  CombineParams cp{};
  cp.part = fp.part;
  cp.nwin = (int64_t)fp.ow * fp.oh;
  cp.ow = fp.ow;
  cp.ngroups = fp.kpad / fp.kg;
  cp.nf = t.n_filters;
  for (int f = 0; f < t.n_filters; ++f) {
    cp.wt[f] = t.weights[f];
    const int32_t* b = &t.boxes[(size_t)f * 4];
    cp.area[f] = (b[2] - b[0]) * (b[3] - b[1]);
  }
  cp.heatmap = a.heatmap;
  cp.best = a.best;
  timing_begin(K_SCORE_COMBINE);
  e = go_combine(cp, s);
  timing_end(K_SCORE_COMBINE);
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
