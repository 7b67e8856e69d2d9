// One-hot integral image of a label map (Sec. 3.1, Supp. S.2) on gfx950.
//
//   P[y][x][j] = #{(x', y') : y' < y, x' < x, label(x', y') = j}
//
// stored channel-last, (H+1) x (W+1) x k int32, exclusive and zero padded.
// The one-hot tensor is never stored: every count comes from the uint8 labels.
//
// The map is cut into 64 x 64 tiles.  P inside tile (r, s) is
//   P[y][x] = corner(r, s) + above(r, x) + left(y, s) + local(y, x)
// where corner counts rows above the tile and columns left of it, above()
// counts rows above the tile in columns [x0, x), left() counts columns left of
// the tile in rows [y0, y) and local() counts inside the tile.  Three kernels:
//   edges : per tile, per-row and per-column label histograms and the tile
//           histogram (small side arrays);
//   prefix: exclusive prefix sums of those histograms across tiles;
//   main  : per tile and chunk of 32 channels, walks its 64 rows: a row of P
//           is the row above plus the per-channel running count along the row
//           (per-channel bit masks of the row's labels and a popcount),
//           streamed out as 16-byte stores of 8 channels per thread.
#include "vqnnf_internal.h"

namespace vqnnf {

namespace {
constexpr int T = kIntTile;   // 64
}

__global__ __launch_bounds__(256) void integral_edges_kernel(IntegralArgs a, int R, int S) {
  extern __shared__ int sh[];   // [64][k]
  const int k = a.k, W = a.W, H = a.H;
  const int s = blockIdx.x, r = blockIdx.y;
  const int x0 = s * T, y0 = r * T;
  const int tw = min(T, W - x0), th = min(T, H - y0);
  const int tid = threadIdx.x;
  for (int i = tid; i < T * k; i += 256) sh[i] = 0;
  __syncthreads();
  for (int i = tid; i < th * tw; i += 256) {
    int dy = i / tw, dx = i % tw;
    int l = a.labels[(int64_t)(y0 + dy) * W + x0 + dx];
    if (l < k) atomicAdd(&sh[dy * k + l], 1);
  }
  __syncthreads();
  for (int i = tid; i < th * k; i += 256) {
    int dy = i / k, j = i % k;
    a.rsh[((int64_t)(y0 + dy) * S + s) * k + j] = sh[i];
  }
  for (int j = tid; j < k; j += 256) {
    int t = 0;
    for (int dy = 0; dy < th; ++dy) t += sh[dy * k + j];
    a.th[((int64_t)r * S + s) * k + j] = t;
  }
  __syncthreads();
  for (int i = tid; i < T * k; i += 256) sh[i] = 0;
  __syncthreads();
  for (int i = tid; i < th * tw; i += 256) {
    int dy = i / tw, dx = i % tw;
    int l = a.labels[(int64_t)(y0 + dy) * W + x0 + dx];
    if (l < k) atomicAdd(&sh[dx * k + l], 1);
  }
  __syncthreads();
  for (int i = tid; i < tw * k; i += 256) {
    int dx = i / k, j = i % k;
    a.cbh[((int64_t)r * W + x0 + dx) * k + j] = sh[i];
  }
}

// Exclusive prefix sums: rsh over strips (per row), cbh over bands (per
// column), th over strips (per band).
__global__ __launch_bounds__(256) void integral_prefix_kernel(IntegralArgs a, int R, int S) {
  const int k = a.k;
  const int64_t n1 = (int64_t)a.H * k, n2 = (int64_t)a.W * k, n3 = (int64_t)R * k;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n1) {
    int64_t y = i / k, j = i % k;
    int acc = 0;
    for (int s = 0; s < S; ++s) {
      int64_t o = (y * S + s) * k + j;
      int v = a.rsh[o];
      a.rsh[o] = acc;
      acc += v;
    }
  } else if (i < n1 + n2) {
    int64_t q = i - n1, x = q / k, j = q % k;
    int acc = 0;
    for (int r = 0; r < R; ++r) {
      int64_t o = ((int64_t)r * a.W + x) * k + j;
      int v = a.cbh[o];
      a.cbh[o] = acc;
      acc += v;
    }
  } else if (i < n1 + n2 + n3) {
    int64_t q = i - n1 - n2, r = q / k, j = q % k;
    int acc = 0;
    for (int s = 0; s < S; ++s) {
      int64_t o = (r * S + s) * k + j;
      int v = a.th[o];
      a.th[o] = acc;
      acc += v;
    }
  }
}

// One block per (tile, chunk of kCK channels); thread t owns pixel column
// t / 4 of the tile and channels [8 (t % 4), +8) of the chunk, so a tile row of
// the chunk is 64 pixels x 32 channels and every thread stores its 8 values
// with one 16-byte (P16) or two 16-byte (int32) stores when the channel
// count is a multiple of 8.
constexpr int kCK = 32;

template <bool P16>
__global__ __launch_bounds__(256) void integral_main_kernel(IntegralArgs a, int R, int S) {
  __shared__ int abv[T][kCK];                    // counts above the tile, then their prefix
  __shared__ unsigned long long masks[2][kCK];   // per channel: the row's label bit mask
  const int k = a.k, W = a.W;
  const int s = blockIdx.x, r = blockIdx.y, j0 = blockIdx.z * kCK;
  const int ck = min(kCK, k - j0);
  const int x0 = s * T, y0 = r * T;
  const int tw = min(T, W - x0), th = min(T, a.H - y0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int dx = tid >> 2, c0 = 8 * (tid & 3);   // pixel column and first channel in the chunk
  const int64_t rowlen = (int64_t)(W + 1) * k;
  // whole 16-byte stores: 8-channel groups start 16-byte aligned
  const bool vec = (k % 8) == 0 && ((uintptr_t)(P16 ? (const void*)a.P16 : (const void*)a.P) % 16) == 0;

  for (int i = tid; i < T * kCK; i += 256) {
    const int x = i / kCK, c = i % kCK;
    abv[x][c] = (x < tw && c < ck) ? a.cbh[((int64_t)r * W + x0 + x) * k + j0 + c] : 0;
  }
  __syncthreads();
  // P[y0][x0 + x + 1][j] = corner + sum_{x' <= x} above[x']
  if (tid < ck) {
    int cnt = 0;
    for (int rr = 0; rr < r; ++rr) cnt += a.th[((int64_t)rr * S + s) * k + j0 + tid];
    for (int x = 0; x < tw; ++x) {
      cnt += abv[x][tid];
      abv[x][tid] = cnt;
    }
  }
  __syncthreads();
  const bool own = dx < tw;
  int V[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) V[c] = abv[dx][c0 + c];
  // the 8 values of this thread at P entry e (channels j0 + c0 ..); threads
  // whose channel group lies past the chunk's channels store nothing
  auto store = [&](int64_t e) {
    if (c0 >= ck) return;
    if (vec) {   // c0 + 8 <= ck: k and so ck are multiples of 8
      if constexpr (P16) {
        uint4 w;
        w.x = (uint32_t)(uint16_t)V[0] | ((uint32_t)(uint16_t)V[1] << 16);
        w.y = (uint32_t)(uint16_t)V[2] | ((uint32_t)(uint16_t)V[3] << 16);
        w.z = (uint32_t)(uint16_t)V[4] | ((uint32_t)(uint16_t)V[5] << 16);
        w.w = (uint32_t)(uint16_t)V[6] | ((uint32_t)(uint16_t)V[7] << 16);
        *(uint4*)(a.P16 + e) = w;
      } else {
        *(int4*)(a.P + e) = make_int4(V[0], V[1], V[2], V[3]);
        *(int4*)(a.P + e + 4) = make_int4(V[4], V[5], V[6], V[7]);
      }
    } else {
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (c0 + c < ck) {
          if constexpr (P16) a.P16[e + c] = (uint16_t)V[c];
          else a.P[e + c] = V[c];
        }
    }
  };
  auto store_zero = [&](int64_t e) {   // zero border entries of the block's channels
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (c0 + c < ck) {
        if constexpr (P16) a.P16[e + c] = 0;
        else a.P[e + c] = 0;
      }
  };
  const int jo = j0 + c0;
  if (r == 0 && own) {
    // row 0 of P: zero
    int Vs[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) { Vs[c] = V[c]; V[c] = 0; }
    store((int64_t)(x0 + dx + 1) * k + jo);
#pragma unroll
    for (int c = 0; c < 8; ++c) V[c] = Vs[c];
    if (s == 0 && dx == 0) store_zero(jo);
  }
  // counts left of the tile in the row (exclusive prefix over tiles), one row ahead
  auto left_of = [&](int y, int (&L)[8]) {
#pragma unroll
    for (int c = 0; c < 8; ++c) L[c] = (c0 + c < ck) ? a.rsh[((int64_t)y * S + s) * k + jo + c] : 0;
  };
  int Lc[8], Ln[8];
  left_of(y0, Lc);
  const unsigned long long below = (2ull << dx) - 1ull;   // columns x0 .. x0 + dx
  for (int dy = 0; dy < th; ++dy) {
    const int y = y0 + dy, buf = dy & 1;
    if (dy + 1 < th) left_of(y + 1, Ln);
    const int l = (lane < tw) ? (int)a.labels[(int64_t)y * W + x0 + lane] - j0 : -1;
#pragma unroll
    for (int i = 0; i < kCK / 4; ++i) {
      const int c = wave * (kCK / 4) + i;
      const unsigned long long m = __ballot(l == c);
      if (lane == 0) masks[buf][c] = m;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 8; ++c) V[c] += Lc[c] + __popcll(masks[buf][c0 + c] & below);
    if (own) store((int64_t)(y + 1) * rowlen + (int64_t)(x0 + dx + 1) * k + jo);
    if (s == 0 && dx == 0) store_zero((int64_t)(y + 1) * rowlen + jo);
#pragma unroll
    for (int c = 0; c < 8; ++c) Lc[c] = Ln[c];
  }
}

namespace {
template <bool P16>
hipError_t go_main(const IntegralArgs& a, int R, int S, hipStream_t st) {
  timing_begin(K_INT_MAIN);
  const dim3 grid((unsigned)S, (unsigned)R, (unsigned)((a.k + kCK - 1) / kCK));
  hipLaunchKernelGGL((integral_main_kernel<P16>), grid, dim3(256), 0, st, a, R, S);
  timing_end(K_INT_MAIN);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_integral(const IntegralArgs& a, hipStream_t st) {
  const int R = (a.H + T - 1) / T, S = (a.W + T - 1) / T;
  size_t lds_e = (size_t)T * a.k * 4;
  if (lds_e > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)integral_edges_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_e);
    if (e != hipSuccess) return e;
  }
  timing_begin(K_INT_EDGE);
  hipLaunchKernelGGL(integral_edges_kernel, dim3(S, R), dim3(256), lds_e, st, a, R, S);
  timing_end(K_INT_EDGE);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t items = ((int64_t)a.H + a.W + R) * a.k;
  timing_begin(K_INT_PREFIX);
  hipLaunchKernelGGL(integral_prefix_kernel, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, st,
                     a, R, S);
  timing_end(K_INT_PREFIX);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return a.P16 ? go_main<true>(a, R, S, st) : go_main<false>(a, R, S, st);
}

}  // namespace vqnnf
