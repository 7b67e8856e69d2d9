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
// The running sum of D^2 is inherently serial and runs on one wave per
// template; the rest is parallel over points, centres and dimensions.
#include "vqnnf_internal.h"

#pragma clang fp contract(off)

namespace vqnnf {

namespace {

constexpr int kKmCK = 16;     // centres per LDS chunk in the assignment
constexpr int kKmTD = 256;    // dimensions per LDS chunk

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

}  // namespace

// k-means++, one draw per launch pair.  km_draw_kernel (one wave per job)
// picks centre ci from the running sum of D^2 (ci = 0: a uniform draw) and
// copies it; km_d2_kernel folds every point's distance to that centre into
// D^2.  The generator state lives in state[0] between launches.
__global__ __launch_bounds__(64) void km_draw_kernel(const KmJob* __restrict__ jobs, int ci) {
  const KmJob j = jobs[blockIdx.x];
  if (ci >= j.k) return;
  __shared__ double chunk_s[64];
  const int lane = threadIdx.x, n = j.l;
  uint64_t rng = ci == 0 ? j.seed : j.state[0];
  const double u = u01(rng);
  int idx = -1;
  if (ci == 0) {
    idx = uniform_index(u, n);
  } else {
    // Strictly in point order: S = the running sum over all points, with the
    // running sum at the end of every chunk of 64 points kept in LDS.  The
    // first chunk whose end exceeds u * S (the sum never decreases, D^2 >= 0)
    // is added once more point by point, from the sum before it, to find the
    // first point above u * S: exactly the additions of one serial running
    // sum.  Buffer loads bounded at n points: lanes past the end read 0; four
    // chunks are in flight while one is added.
    const __amdgpu_buffer_rsrc_t d2r = __builtin_amdgcn_make_buffer_rsrc(j.d2, (short)0, n * 8, 0x00020000);
    auto ld = [&](int p) -> double {
      return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(d2r, (uint32_t)p * 8u, 0, 0));
    };
    // a chunk's values go through LDS and are all read (broadcast) into
    // registers before the dependent chain of additions
    auto add_chunk = [&](double v, int cnt, double r) -> double {
      chunk_s[lane] = v;
      if (cnt >= 64) {
        double w[64];
#pragma unroll
        for (int i = 0; i < 64; ++i) w[i] = chunk_s[i];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < 64; ++i) r = r + w[i];
      } else {
        for (int i = 0; i < cnt; ++i) r = r + chunk_s[i];
      }
      return r;
    };
    // templates have at most 255 x 255 points: 1017 chunks
    constexpr int kEnds = 1024;
    __shared__ double ends_s[kEnds];
    const int nc = (n + 63) / 64;
    const bool keep = nc <= kEnds;
    double run = 0.0;
    {
      double q0 = ld(lane), q1 = ld(64 + lane), q2 = ld(128 + lane), q3 = ld(192 + lane);
      for (int base = 0; base < n; base += 256) {
        const int c = base / 64;
        run = add_chunk(q0, n - base, run);
        if (keep && lane == 0 && c < nc) ends_s[c] = run;
        q0 = ld(base + 256 + lane);
        run = add_chunk(q1, n - base - 64, run);
        if (keep && lane == 0 && c + 1 < nc) ends_s[c + 1] = run;
        q1 = ld(base + 320 + lane);
        run = add_chunk(q2, n - base - 128, run);
        if (keep && lane == 0 && c + 2 < nc) ends_s[c + 2] = run;
        q2 = ld(base + 384 + lane);
        run = add_chunk(q3, n - base - 192, run);
        if (keep && lane == 0 && c + 3 < nc) ends_s[c + 3] = run;
        q3 = ld(base + 448 + lane);
      }
    }
    __syncthreads();
    const double total = run;
    if (total == 0.0) {
      idx = uniform_index(u, n);
    } else {
      const double target = u * total;
      int hit = -1;                      // first chunk whose end exceeds the target
      double before = 0.0;               // running sum before that chunk
      if (keep) {
        for (int c0 = 0; c0 < nc && hit < 0; c0 += 64) {
          const int c = c0 + lane;
          const unsigned long long b = __ballot(c < nc && ends_s[c < nc ? c : 0] > target);
          if (b) hit = c0 + __ffsll((long long)b) - 1;
        }
        if (hit > 0) before = ends_s[hit - 1];
        if (hit >= 0) hit *= 64;
      } else {
        // more chunks than kept: the running sum again, chunk by chunk
        run = 0.0;
        for (int base = 0; base < n; base += 64) {
          const double r = add_chunk(ld(base + lane), n - base, run);
          if (r > target) { hit = base; before = run; break; }
          run = r;
        }
      }
      if (hit >= 0) {
        double r = before;
        const int nb = min(64, n - hit);
        chunk_s[lane] = ld(hit + lane);
        for (int i = 0; i < nb; ++i) {
          r = r + chunk_s[i];
          if (r > target) { idx = hit + i; break; }
        }
      }
      if (idx < 0) {
        // no running sum exceeded u * S: the last point with D^2 > 0
        int last = -1;
        for (int p = lane; p < n; p += 64)
          if (j.d2[p] > 0.0) last = p;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) last = max(last, __shfl_xor(last, m));
        idx = last;
      }
    }
  }
  for (int t = lane; t < j.D; t += 64) j.c[(size_t)ci * j.D + t] = (double)j.x[(size_t)idx * j.D + t];
  if (lane == 0) j.state[0] = rng;
}

// D^2 of every point to centre ci, folded in by minimum (ci = 0: written).
// Thread per point; the centre is staged in LDS in chunks of kKmTD.
__global__ __launch_bounds__(256) void km_d2_kernel(const KmJob* __restrict__ jobs, int ci) {
  const KmJob j = jobs[blockIdx.y];
  if (ci >= j.k - 1 || (int64_t)blockIdx.x * 256 >= j.l) return;   // uniform per block
  __shared__ double cs[kKmTD];
  const int n = j.l, D = j.D;
  const int p = blockIdx.x * 256 + threadIdx.x;
  const float* xtp = j.xt + min(p, n - 1);       // dimension-major: coalesced across the wave
  double acc = 0.0;
  for (int t0 = 0; t0 < D; t0 += kKmTD) {
    const int tn = min(kKmTD, D - t0);
    __syncthreads();
    for (int t = threadIdx.x; t < tn; t += 256) cs[t] = j.c[(size_t)ci * D + t0 + t];
    __syncthreads();
#pragma unroll 8
    for (int t = 0; t < tn; ++t) {
      const double diff = (double)xtp[(int64_t)(t0 + t) * n] - cs[t];
      const double sq = diff * diff;
      acc = acc + sq;
    }
  }
  if (p < n) j.d2[p] = ci == 0 ? acc : (acc < j.d2[p] ? acc : j.d2[p]);
}

// Distances of a block of 256 points to one chunk of kKmCK centres (FP64
// centres, or the FP32 codebook when from_f32 is set); writes the chunk's
// nearest centre (lowest index on ties) and its distance.  The centres are
// staged dimension-major (one dimension's kKmCK values contiguous, read as
// broadcast 16-byte words); each thread requests its point's values 16
// dimensions ahead of the ones it is accumulating.
__global__ __launch_bounds__(256) void km_assign_kernel(const KmJob* __restrict__ jobs, int from_f32) {
  const KmJob& j = jobs[blockIdx.z];
  const int n = j.l, D = j.D, k = j.k;
  const int c0 = blockIdx.y * kKmCK;
  if (c0 >= k || (int64_t)blockIdx.x * 256 >= n) return;   // uniform per block
  const int nc = min(kKmCK, k - c0);
  __shared__ double cs[kKmTD][kKmCK];
  const int p = blockIdx.x * 256 + threadIdx.x;
  const float* xtp = j.xt + min(p, n - 1);       // dimension-major: coalesced across the wave
  double acc[kKmCK];
#pragma unroll
  for (int i = 0; i < kKmCK; ++i) acc[i] = 0.0;
  constexpr int PF = 16;                         // dimensions per prefetch group
  for (int t0 = 0; t0 < D; t0 += kKmTD) {
    const int tn = min(kKmTD, D - t0);
    __syncthreads();
    for (int e = threadIdx.x; e < kKmCK * kKmTD; e += 256) {
      const int t = e / kKmCK, ci = e % kKmCK;
      double v = 0.0;
      if (ci < nc && t < tn)
        v = from_f32 ? (double)j.c32[(size_t)(c0 + ci) * D + t0 + t] : j.c[(size_t)(c0 + ci) * D + t0 + t];
      cs[t][ci] = v;
    }
    __syncthreads();
    // a global-address-space pointer: the point values are read with global
    // loads (only the vector-memory counter), so the waits for them leave
    // the LDS reads of the centres alone
    typedef __attribute__((address_space(1))) const float gfloat;
    gfloat* xq = (gfloat*)(xtp + (int64_t)t0 * n);
    float xa[PF], xb[PF];
    auto ldx = [&](float (&dst)[PF], int g) {
#pragma unroll
      for (int u = 0; u < PF; ++u) dst[u] = xq[(int64_t)min(g + u, tn - 1) * n];   // past tn: unused
    };
    // dimensions t0 + g .. t0 + g + PF - 1, in order
    auto comp = [&](const float (&src)[PF], int g) {
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        if (g + u >= tn) break;
        const double xv = (double)src[u];
#pragma unroll
        for (int i = 0; i < kKmCK; ++i) {
          const double diff = xv - cs[g + u][i];
          const double sq = diff * diff;
          acc[i] = acc[i] + sq;
        }
      }
    };
    ldx(xa, 0);
    for (int g = 0; g < tn; g += 2 * PF) {
      ldx(xb, g + PF);
      comp(xa, g);
      ldx(xa, g + 2 * PF);
      comp(xb, g + PF);
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
__global__ __launch_bounds__(1024) void km_sort_kernel(const KmJob* __restrict__ jobs) {
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
// cluster's points in point order, divided by the count.  Groups of G points:
// the point indices are requested one group ahead of their values and the
// values one group ahead of their additions (global loads: only the
// vector-memory counter), so each group waits for one memory round trip.
__global__ __launch_bounds__(256) void km_update_kernel(const KmJob* __restrict__ jobs) {
  const KmJob& j = jobs[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)j.k * j.D) return;
  const int D = j.D;
  const int c = (int)(e / D), t = (int)(e % D);
  const int b = j.start[c], nb = j.start[c + 1] - b;
  if (nb == 0) return;                     // empty cluster keeps its centre
  typedef __attribute__((address_space(1))) const int gint;
  typedef __attribute__((address_space(1))) const float gfloat;
  gint* ip = (gint*)(j.idx + b);
  gfloat* xp = (gfloat*)(j.x + t);
  constexpr int G = 32;
  int ia[G];                               // indices of the next group
  float va[G], vb[G];                      // values of this group and the next
  // past the cluster's end: its last point again (read, never added)
#pragma unroll
  for (int q = 0; q < G; ++q) ia[q] = ip[min(q, nb - 1)];
#pragma unroll
  for (int q = 0; q < G; ++q) va[q] = xp[(size_t)ia[q] * D];
#pragma unroll
  for (int q = 0; q < G; ++q) ia[q] = ip[min(G + q, nb - 1)];
  double s = 0.0;
  for (int m = 0; m < nb; m += G) {
#pragma unroll
    for (int q = 0; q < G; ++q) vb[q] = xp[(size_t)ia[q] * D];
#pragma unroll
    for (int q = 0; q < G; ++q) ia[q] = ip[min(m + 2 * G + q, nb - 1)];
#pragma unroll
    for (int q = 0; q < G; ++q)
      if (m + q < nb) s = s + (double)va[q];
#pragma unroll
    for (int q = 0; q < G; ++q) va[q] = vb[q];
  }
  j.c[e] = s / (double)nb;
}

// Dimension-major copy of the points for the distance kernels.
__global__ __launch_bounds__(256) void km_transpose_kernel(const KmJob* __restrict__ jobs) {
  const KmJob& j = jobs[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)j.l * j.D) return;
  const int t = (int)(e / j.l), p = (int)(e % j.l);
  j.xt[e] = j.x[(size_t)p * j.D + t];
}

__global__ __launch_bounds__(256) void km_round_kernel(const KmJob* __restrict__ jobs) {
  const KmJob& j = jobs[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < (int64_t)j.k * j.D) j.c32[e] = (float)j.c[e];
}

hipError_t launch_kmeans(const KmJob* d_jobs, const std::vector<KmJob>& jobs, int iters, hipStream_t s) {
  const int nj = (int)jobs.size();
  int max_l = 1, max_k = 1;
  int64_t max_kd = 1, max_ld = 1;
  for (const KmJob& j : jobs) {
    max_l = std::max(max_l, j.l);
    max_k = std::max(max_k, j.k);
    max_kd = std::max(max_kd, (int64_t)j.k * j.D);
    max_ld = std::max(max_ld, (int64_t)j.l * j.D);
  }
  const dim3 ga((unsigned)((max_l + 255) / 256), (unsigned)((max_k + kKmCK - 1) / kKmCK), (unsigned)nj);
  const dim3 gu((unsigned)((max_kd + 255) / 256), (unsigned)nj);
  timing_begin(K_KMEANS);
  hipLaunchKernelGGL(km_transpose_kernel, dim3((unsigned)((max_ld + 255) / 256), (unsigned)nj), dim3(256), 0, s,
                     d_jobs);
  const dim3 gd((unsigned)((max_l + 255) / 256), (unsigned)nj);
  for (int ci = 0; ci < max_k; ++ci) {
    hipLaunchKernelGGL(km_draw_kernel, dim3(nj), dim3(64), 0, s, d_jobs, ci);
    if (ci + 1 < max_k) hipLaunchKernelGGL(km_d2_kernel, gd, dim3(256), 0, s, d_jobs, ci);
  }
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
