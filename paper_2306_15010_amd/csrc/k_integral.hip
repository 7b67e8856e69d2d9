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
//   main  : per tile, walks its 64 rows: a row of P is the row above plus the
//           per-channel running count along the row (per-channel bit masks of
//           the row's labels and a popcount), streamed out with coalesced
//           stores (one tile row of P is one contiguous block of memory).
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

// VPT: values of one tile row held per thread, ceil(64 * k / 256).
template <int VPT>
__global__ __launch_bounds__(256) void integral_main_kernel(IntegralArgs a, int R, int S) {
  extern __shared__ int smem[];
  const int k = a.k, W = a.W, H = a.H;
  const int s = blockIdx.x, r = blockIdx.y;
  const int x0 = s * T, y0 = r * T;
  const int tw = min(T, W - x0), th = min(T, H - y0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int* abv = smem;                                              // [64][k]
  unsigned long long* masks = (unsigned long long*)(smem + T * k);  // [2][k]
  int* left = (int*)(masks + 2 * k);                            // [2][k]
  const int64_t rowlen = (int64_t)(W + 1) * k;

  for (int i = tid; i < tw * k; i += 256) {
    int dx = i / k, j = i % k;
    abv[i] = a.cbh[((int64_t)r * W + x0 + dx) * k + j];
  }
  __syncthreads();
  // P[y0][x0 + dx + 1][j] = corner + sum_{x' <= dx} above[x']
  for (int j = tid; j < k; j += 256) {
    int c = 0;
    for (int rr = 0; rr < r; ++rr) c += a.th[((int64_t)rr * S + s) * k + j];
    for (int dx = 0; dx < tw; ++dx) {
      c += abv[dx * k + j];
      abv[dx * k + j] = c;
    }
  }
  __syncthreads();
  int V[VPT];
  int vdx[VPT], vj[VPT];
#pragma unroll
  for (int i = 0; i < VPT; ++i) {
    int f = tid + 256 * i;
    vdx[i] = f / k;
    vj[i] = f % k;
    V[i] = (f < tw * k) ? abv[f] : 0;
  }
  // 32-bit P, or P mod 2^16 (differences of taps still give exact counts
  // below 2^16 in wrapping 16-bit arithmetic)
  auto put = [&](int64_t i, int v) {
    if (a.P16) a.P16[i] = (uint16_t)v;
    else a.P[i] = v;
  };
  if (r == 0) {
#pragma unroll
    for (int i = 0; i < VPT; ++i)
      if (tid + 256 * i < tw * k) put((int64_t)(x0 + vdx[i] + 1) * k + vj[i], 0);
    if (s == 0)
      for (int j = tid; j < k; j += 256) put(j, 0);
  }
  // per-channel slice of the mask computation for this wave
  const int jw0 = (k * wave) / 4, jw1 = (k * (wave + 1)) / 4;
  for (int dy = 0; dy < th; ++dy) {
    const int y = y0 + dy;
    const int buf = dy & 1;
    const int l = (lane < tw) ? (int)a.labels[(int64_t)y * W + x0 + lane] : 0xFFFF;
    for (int j = jw0; j < jw1; ++j) {
      unsigned long long m = __ballot(l == j);
      if (lane == 0) masks[buf * k + j] = m;
    }
    for (int j = tid; j < k; j += 256) left[buf * k + j] = a.rsh[((int64_t)y * S + s) * k + j];
    __syncthreads();
    const int64_t prow = (int64_t)(y + 1) * rowlen + (int64_t)(x0 + 1) * k;
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      if (tid + 256 * i < tw * k) {
        const unsigned long long below = (2ull << vdx[i]) - 1ull;
        const int cnt = __popcll(masks[buf * k + vj[i]] & below);
        V[i] += left[buf * k + vj[i]] + cnt;
        put(prow + tid + 256 * i, V[i]);
      }
    }
    if (s == 0)
      for (int j = tid; j < k; j += 256) put((int64_t)(y + 1) * rowlen + j, 0);
  }
}

namespace {
template <int VPT>
hipError_t go_main(const IntegralArgs& a, int R, int S, hipStream_t st) {
  size_t lds = (size_t)T * a.k * 4 + 2 * (size_t)a.k * 8 + 2 * (size_t)a.k * 4;
  auto kern = integral_main_kernel<VPT>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  timing_begin(K_INT_MAIN);
  hipLaunchKernelGGL(kern, dim3(S, R), dim3(256), lds, st, a, R, S);
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
  const int vpt = (T * a.k + 255) / 256;
  if (vpt <= 1) return go_main<1>(a, R, S, st);
  if (vpt <= 2) return go_main<2>(a, R, S, st);
  if (vpt <= 4) return go_main<4>(a, R, S, st);
  if (vpt <= 8) return go_main<8>(a, R, S, st);
  if (vpt <= 16) return go_main<16>(a, R, S, st);
  if (vpt <= 32) return go_main<32>(a, R, S, st);
  return go_main<64>(a, R, S, st);
}

}  // namespace vqnnf
