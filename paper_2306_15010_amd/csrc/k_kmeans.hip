// Template codebooks on the GPU: seeded k-means++ and Lloyd iterations in
// FP64 (Sec. 3.1; Sec. 4 "K-means computation"; Sec. 5.2 "Codebook and NNF
// Generation"), then the template's NNF against the FP32-rounded codebook.
//
// Every floating-point operation is the same IEEE FP64 operation, in the same
// order, as the host definition the library's CPU path also follows, so the
// codebook and labels are bit-identical to it:
//   * squared distance d(p, c) = sum_t (x_pt - c_t)^2, sequential in t from 0,
//     subtract, multiply and add rounded separately (no contraction in this
//     file);
//   * k-means++: the first centre is point min(floor(u * n), n - 1); each next
//     centre is the first point whose sequential running sum of D^2 exceeds
//     u * S (S = the full sequential sum; if none does, the last point with
//     D^2 > 0; if S = 0, a uniform draw), with u = (splitmix64 >> 11) * 2^-53;
//     D^2 keeps the minimum over the chosen centres;
//   * Lloyd: each point goes to its nearest centre (lowest index on ties);
//     each centre becomes the sequential sum of its points in point order
//     divided by their count; an empty cluster keeps its centre.
// The running sum of D^2 is inherently serial and runs on one lane; the rest
// is parallel over points, centres and dimensions.
#include "vqnnf_internal.h"

#pragma clang fp contract(off)

namespace vqnnf {

namespace {

constexpr int kKmCK = 16;     // centres per LDS chunk in the assignment
constexpr int kKmTD = 256;    // dimensions per LDS chunk
constexpr int kKmInitThreads = 1024;

__device__ __forceinline__ uint64_t splitmix_next(uint64_t& s) {
  s += 0x9E3779B97F4A7C15ull;
  uint64_t z = s;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double u01(uint64_t& s) {
  return (double)(splitmix_next(s) >> 11) * 0x1.0p-53;
}

__device__ __forceinline__ int uniform_index(double u, int n) {
  const double f = floor(u * (double)n);
  return f >= (double)(n - 1) ? n - 1 : (int)f;
}

// d(x_p, c) for one point against a centre staged in LDS in chunks of kKmTD.
__device__ double sqdist_lds(const float* xp, const double* cs, int t0, int tn, double acc) {
  for (int t = 0; t < tn; ++t) {
    const double diff = (double)xp[t0 + t] - cs[t];
    const double sq = diff * diff;
    acc = acc + sq;
  }
  return acc;
}

// D^2 of every point to centre `ci` (already in c), folded into d2 by minimum
// (first centre: written).  Whole block.
__device__ void km_update_d2(const KmJob& j, int ci, bool first, double* cs) {
  double acc[8];
  const int n = j.l, D = j.D;
  // points handled by this thread: p = tid + i * blockDim, up to 8 per pass
  for (int p0 = 0; p0 < n; p0 += 8 * kKmInitThreads) {
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = 0.0;
    for (int t0 = 0; t0 < D; t0 += kKmTD) {
      const int tn = min(kKmTD, D - t0);
      __syncthreads();
      for (int t = threadIdx.x; t < tn; t += blockDim.x) cs[t] = j.c[(size_t)ci * D + t0 + t];
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int p = p0 + threadIdx.x + i * kKmInitThreads;
        if (p < n) acc[i] = sqdist_lds(j.x + (size_t)p * D, cs, t0, tn, acc[i]);
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int p = p0 + threadIdx.x + i * kKmInitThreads;
      if (p < n) j.d2[p] = first ? acc[i] : (acc[i] < j.d2[p] ? acc[i] : j.d2[p]);
    }
  }
  __syncthreads();
}

__device__ void copy_point_to_centre(const KmJob& j, int p, int ci) {
  for (int t = threadIdx.x; t < j.D; t += blockDim.x)
    j.c[(size_t)ci * j.D + t] = (double)j.x[(size_t)p * j.D + t];
  __syncthreads();
}

}  // namespace

// k-means++ seeding, one block per job.
__global__ __launch_bounds__(kKmInitThreads) void km_init_kernel(const KmJob* jobs) {
  const KmJob& j = jobs[blockIdx.x];
  __shared__ double cs[kKmTD];
  __shared__ double sh_total, sh_u;
  __shared__ int sh_idx;
  __shared__ int red[kKmInitThreads / 64];
  uint64_t rng = j.seed;                 // every thread steps the same stream
  const int n = j.l;
  const int first = uniform_index(u01(rng), n);
  copy_point_to_centre(j, first, 0);
  km_update_d2(j, 0, true, cs);
  for (int ci = 1; ci < j.k; ++ci) {
    if (threadIdx.x == 0) {
      double run = 0.0;
      for (int p = 0; p < n; ++p) {
        run = run + j.d2[p];
        j.csum[p] = run;
      }
      sh_total = run;
    }
    const double u = u01(rng);
    __syncthreads();
    const double total = sh_total;
    int idx;
    if (total == 0.0) {
      idx = uniform_index(u, n);
    } else {
      const double target = u * total;
      // first p with csum[p] > target; else the last p with d2[p] > 0
      int best = 0x7FFFFFFF, last = -1;
      for (int p = threadIdx.x; p < n; p += blockDim.x) {
        if (j.csum[p] > target && p < best) best = p;
        if (j.d2[p] > 0.0) last = p;
      }
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) {
        best = min(best, __shfl_xor(best, m));
        last = max(last, __shfl_xor(last, m));
      }
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
      __syncthreads();
      if (threadIdx.x == 0) {
        int b = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) b = min(b, red[w]);
        sh_idx = b;
      }
      __syncthreads();
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = last;
      __syncthreads();
      if (threadIdx.x == 0 && sh_idx == 0x7FFFFFFF) {
        int l2 = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) l2 = max(l2, red[w]);
        sh_idx = l2;
      }
      __syncthreads();
      idx = sh_idx;
    }
    copy_point_to_centre(j, idx, ci);
    km_update_d2(j, ci, false, cs);
  }
}

// Distances of a block of 256 points to one chunk of kKmCK centres (FP64
// centres, or the FP32 codebook when c32in is set); writes the chunk's
// nearest centre (lowest index on ties) and its distance.
__global__ __launch_bounds__(256) void km_assign_kernel(const KmJob* jobs, int from_f32) {
  const KmJob& j = jobs[blockIdx.z];
  const int n = j.l, D = j.D, k = j.k;
  const int c0 = blockIdx.y * kKmCK;
  if (c0 >= k || (int64_t)blockIdx.x * 256 >= n) return;   // uniform per block
  const int nc = min(kKmCK, k - c0);
  __shared__ double cs[kKmCK][kKmTD];
  const int p = blockIdx.x * 256 + threadIdx.x;
  const float* xp = j.x + (size_t)min(p, n - 1) * D;
  double acc[kKmCK];
#pragma unroll
  for (int i = 0; i < kKmCK; ++i) acc[i] = 0.0;
  for (int t0 = 0; t0 < D; t0 += kKmTD) {
    const int tn = min(kKmTD, D - t0);
    __syncthreads();
    for (int e = threadIdx.x; e < kKmCK * kKmTD; e += 256) {
      const int ci = e / kKmTD, t = e % kKmTD;
      double v = 0.0;
      if (ci < nc && t < tn)
        v = from_f32 ? (double)j.c32[(size_t)(c0 + ci) * D + t0 + t] : j.c[(size_t)(c0 + ci) * D + t0 + t];
      cs[ci][t] = v;
    }
    __syncthreads();
    for (int t = 0; t < tn; ++t) {
      const double xv = (double)xp[t0 + t];
#pragma unroll
      for (int i = 0; i < kKmCK; ++i) {
        const double diff = xv - cs[i][t];
        const double sq = diff * diff;
        acc[i] = acc[i] + sq;
      }
    }
  }
  if (p < n) {
    double best = acc[0];
    int bi = 0;
#pragma unroll
    for (int i = 1; i < kKmCK; ++i)
      if (i < nc && acc[i] < best) { best = acc[i]; bi = i; }
    j.pdist[(size_t)blockIdx.y * n + p] = best;
    j.pidx[(size_t)blockIdx.y * n + p] = (uint8_t)(c0 + bi);
  }
}

// Labels from the per-chunk nearest centres (chunks in index order, strict <
// keeps the lowest index), then a stable counting sort of the points by
// label: idx lists every cluster's points in increasing point order.
__global__ __launch_bounds__(1024) void km_sort_kernel(const KmJob* jobs) {
  const KmJob& j = jobs[blockIdx.x];
  const int n = j.l, k = j.k;
  const int nch = (k + kKmCK - 1) / kKmCK;
  constexpr int NW = 16;                     // waves, one contiguous segment each
  __shared__ int cnt[NW][kMaxK];
  __shared__ int run[NW][kMaxK];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < NW * kMaxK; i += blockDim.x) (&cnt[0][0])[i] = 0;
  __syncthreads();
  for (int p = threadIdx.x; p < n; p += blockDim.x) {
    double best = j.pdist[p];
    int bi = j.pidx[p];
    for (int c = 1; c < nch; ++c) {
      const double d = j.pdist[(size_t)c * n + p];
      if (d < best) { best = d; bi = j.pidx[(size_t)c * n + p]; }
    }
    j.lab[p] = (uint8_t)bi;
  }
  __syncthreads();
  const int seg = (n + NW - 1) / NW;
  const int s0 = w * seg, s1 = min(n, s0 + seg);
  for (int p = s0 + lane; p < s1; p += 64) atomicAdd(&cnt[w][j.lab[p]], 1);
  __syncthreads();
  if (threadIdx.x < k) {
    // start of cluster c, and of each segment's first point of it
    const int c = threadIdx.x;
    int before = 0;
    for (int c2 = 0; c2 < c; ++c2)
      for (int w2 = 0; w2 < NW; ++w2) before += cnt[w2][c2];
    j.start[c] = before;
    int r = before;
    for (int w2 = 0; w2 < NW; ++w2) {
      run[w2][c] = r;
      r += cnt[w2][c];
    }
    if (c == k - 1) j.start[k] = r;
  }
  __syncthreads();
  // each wave scatters its segment in order, 64 points at a time
  for (int b = s0; b < s1; b += 64) {
    const int p = b + lane;
    const bool act = p < s1;
    int lb = act ? (int)j.lab[p] : -1;
    uint64_t todo = __ballot(act);
    while (todo) {
      const int leader = __builtin_amdgcn_readfirstlane(__ffsll((long long)todo) - 1);
      const int lv = __shfl(lb, leader);
      const uint64_t m = __ballot(act && lb == lv);
      if (act && lb == lv) {
        const int rank = __popcll(m & ((1ull << lane) - 1ull));
        j.idx[run[w][lv] + rank] = p;
      }
      if (lane == leader) run[w][lv] += __popcll(m);
      todo &= ~m;
      __builtin_amdgcn_wave_barrier();
    }
  }
}

// New centres: thread per (cluster, dimension), sequential sum of the
// cluster's points in point order, divided by the count.
__global__ __launch_bounds__(256) void km_update_kernel(const KmJob* jobs) {
  const KmJob& j = jobs[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)j.k * j.D) return;
  const int c = (int)(e / j.D), t = (int)(e % j.D);
  const int b = j.start[c], nb = j.start[c + 1] - b;
  if (nb == 0) return;                     // empty cluster keeps its centre
  double s = 0.0;
  for (int m = 0; m < nb; ++m) s = s + (double)j.x[(size_t)j.idx[b + m] * j.D + t];
  j.c[e] = s / (double)nb;
}

__global__ __launch_bounds__(256) void km_round_kernel(const KmJob* jobs) {
  const KmJob& j = jobs[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < (int64_t)j.k * j.D) j.c32[e] = (float)j.c[e];
}

hipError_t launch_kmeans(const KmJob* d_jobs, const std::vector<KmJob>& jobs, int iters, hipStream_t s) {
  const int nj = (int)jobs.size();
  int max_l = 1, max_k = 1;
  int64_t max_kd = 1;
  for (const KmJob& j : jobs) {
    max_l = std::max(max_l, j.l);
    max_k = std::max(max_k, j.k);
    max_kd = std::max(max_kd, (int64_t)j.k * j.D);
  }
  const dim3 ga((unsigned)((max_l + 255) / 256), (unsigned)((max_k + kKmCK - 1) / kKmCK), (unsigned)nj);
  const dim3 gu((unsigned)((max_kd + 255) / 256), (unsigned)nj);
  timing_begin(K_KMEANS);
  hipLaunchKernelGGL(km_init_kernel, dim3(nj), dim3(kKmInitThreads), 0, s, d_jobs);
  for (int it = 0; it < iters; ++it) {
    hipLaunchKernelGGL(km_assign_kernel, ga, dim3(256), 0, s, d_jobs, 0);
    hipLaunchKernelGGL(km_sort_kernel, dim3(nj), dim3(1024), 0, s, d_jobs);
    hipLaunchKernelGGL(km_update_kernel, gu, dim3(256), 0, s, d_jobs);
  }
  hipLaunchKernelGGL(km_round_kernel, gu, dim3(256), 0, s, d_jobs);
  // the template's NNF against the FP32 codebook
  hipLaunchKernelGGL(km_assign_kernel, ga, dim3(256), 0, s, d_jobs, 1);
  hipLaunchKernelGGL(km_sort_kernel, dim3(nj), dim3(1024), 0, s, d_jobs);
  timing_end(K_KMEANS);
  return hipGetLastError();
}

}  // namespace vqnnf
