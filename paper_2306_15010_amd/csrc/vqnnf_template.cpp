// Host-side template preparation: k-means codebook, template NNF, template
// representation R(tau), and the device-ready tables (matrix-core fragments,
// codeword norms, error-bound constants).
//
// Floating-point contract: every FP64 distance is sum_t (q_t - c_t)^2 taken
// sequentially in t from 0, with separate subtract, multiply and add.  This
// file is compiled with -ffp-contract=off so no FMA is formed.
#pragma clang fp contract(off)

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

#include "vqnnf_internal.h"

namespace vqnnf {

namespace {

template <typename F>
void parallel_for(int64_t n, F&& f, int64_t min_n = 4096) {
  unsigned hw = std::thread::hardware_concurrency();
  int nt = (int)std::max(1u, std::min(hw ? hw : 1u, 32u));
  if (n < min_n || nt == 1) {
    f((int64_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  int64_t per = (n + nt - 1) / nt;
  for (int i = 0; i < nt; ++i) {
    int64_t b = i * per, e = std::min(n, b + per);
    if (b >= e) break;
    th.emplace_back([&, b, e] { f(b, e); });
  }
  for (auto& t : th) t.join();
}

struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double u01() { return (double)(next() >> 11) * 0x1.0p-53; }
};

int uniform_index(double u, int64_t n) {
  int64_t i = (int64_t)std::floor(u * (double)n);
  return (int)std::min<int64_t>(i, n - 1);
}

// Sequential FP64 squared distance.
inline double sqdist(const double* x, const double* c, int D) {
  double acc = 0.0;
  for (int t = 0; t < D; ++t) {
    double d = x[t] - c[t];
    double sq = d * d;
    acc = acc + sq;
  }
  return acc;
}

// dist[p][j] for all points and centres; centres given as [k][D].
void all_distances(const std::vector<double>& x, int64_t n, const std::vector<double>& c, int k,
                   int D, std::vector<double>& out) {
  out.resize((size_t)n * k);
  // transpose centres to [D][k] so the inner loop runs over centres: every
  // centre keeps its own sequential sum over t
  std::vector<double> ct((size_t)D * k);
  for (int j = 0; j < k; ++j)
    for (int t = 0; t < D; ++t) ct[(size_t)t * k + j] = c[(size_t)j * D + t];
  parallel_for(n, [&](int64_t b, int64_t e) {
    std::vector<double> acc(k);
    for (int64_t p = b; p < e; ++p) {
      const double* xp = &x[(size_t)p * D];
      std::fill(acc.begin(), acc.end(), 0.0);
      for (int t = 0; t < D; ++t) {
        const double xv = xp[t];
        const double* cr = &ct[(size_t)t * k];
        for (int j = 0; j < k; ++j) {
          double d = xv - cr[j];
          double sq = d * d;
          acc[j] = acc[j] + sq;
        }
      }
      std::memcpy(&out[(size_t)p * k], acc.data(), sizeof(double) * k);
    }
  });
}

void argmin_rows(const std::vector<double>& d, int64_t n, int k, std::vector<int>& lab) {
  lab.resize(n);
  for (int64_t p = 0; p < n; ++p) {
    const double* r = &d[(size_t)p * k];
    int best = 0;
    for (int j = 1; j < k; ++j)
      if (r[j] < r[best]) best = j;
    lab[p] = best;
  }
}

}  // namespace

// k-means++ seeding then `iters` Lloyd iterations (Sec. 3.1), FP64.
std::vector<double> kmeans_host(const std::vector<double>& x, int64_t n, int D, int k, int iters,
                                uint64_t seed) {
  SplitMix64 rng{seed};
  std::vector<double> c((size_t)k * D);
  int first = uniform_index(rng.u01(), n);
  std::copy(&x[(size_t)first * D], &x[(size_t)first * D] + D, &c[0]);
  std::vector<double> d2(n), csum(n);
  parallel_for(n, [&](int64_t b, int64_t e) {
    for (int64_t p = b; p < e; ++p) d2[p] = sqdist(&x[(size_t)p * D], &c[0], D);
  });
  for (int i = 1; i < k; ++i) {
    double run = 0.0;
    for (int64_t p = 0; p < n; ++p) {
      run = run + d2[p];
      csum[p] = run;
    }
    double total = csum[n - 1];
    double u = rng.u01();
    int64_t idx;
    if (total == 0.0) {
      idx = uniform_index(u, n);
    } else {
      double target = u * total;
      idx = -1;
      for (int64_t p = 0; p < n; ++p)
        if (csum[p] > target) { idx = p; break; }
      if (idx < 0)
        for (int64_t p = n - 1; p >= 0; --p)
          if (d2[p] > 0.0) { idx = p; break; }
    }
    double* ci = &c[(size_t)i * D];
    std::copy(&x[(size_t)idx * D], &x[(size_t)idx * D] + D, ci);
    parallel_for(n, [&](int64_t b, int64_t e) {
      for (int64_t p = b; p < e; ++p) {
        double dn = sqdist(&x[(size_t)p * D], ci, D);
        if (dn < d2[p]) d2[p] = dn;
      }
    });
  }
  std::vector<double> dist;
  std::vector<int> lab;
  std::vector<double> sum(D);
  for (int it = 0; it < iters; ++it) {
    all_distances(x, n, c, k, D, dist);
    argmin_rows(dist, n, k, lab);
    // per-cluster sequential sums in point order
    std::vector<double> sums((size_t)k * D, 0.0);
    std::vector<int64_t> cnt(k, 0);
    for (int64_t p = 0; p < n; ++p) {
      int j = lab[p];
      double* s = &sums[(size_t)j * D];
      const double* xp = &x[(size_t)p * D];
      for (int t = 0; t < D; ++t) s[t] = s[t] + xp[t];
      cnt[j] += 1;
    }
    for (int j = 0; j < k; ++j) {
      if (cnt[j] == 0) continue;
      double nj = (double)cnt[j];
      for (int t = 0; t < D; ++t) c[(size_t)j * D + t] = sums[(size_t)j * D + t] / nj;
    }
  }
  return c;
}

// FP64 nearest codeword (lowest index on ties) of every point.
std::vector<int> assign_host(const std::vector<double>& x, int64_t n, int D,
                             const std::vector<double>& c, int k) {
  std::vector<double> dist;
  std::vector<int> lab;
  all_distances(x, n, c, k, D, dist);
  argmin_rows(dist, n, k, lab);
  return lab;
}

AssignGeom make_assign_geom(int k, int D) {
  AssignGeom g{};
  // codeword blocks of 16, rounded to the kernel instances (1, 2, 3, 4, 8, 16)
  g.kb = (k + 15) / 16;
  if (g.kb > 4 && g.kb <= 8) g.kb = 8;
  if (g.kb > 8) g.kb = 16;
  g.kpad = 16 * g.kb;
  int d32 = ((D + 31) / 32) * 32;
  // one K-step (32 elements) per load group: with the next group's query
  // and codebook fragments in flight, larger groups overflow the register
  // budget of 8 waves per CU
  g.s_bf16 = 1;
  // an even number of groups: the kernel alternates two query buffers
  g.d_pad_bf16 = ((D + 63) / 64) * 64;
  int d16 = ((D + 15) / 16) * 16;
  g.e_f32 = (g.kb < 8 && d16 % 32 == 0) ? 8 : 4;
  g.d_pad_f32 = d16;
  return g;
}

namespace {

uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  uint32_t lsb = (u >> 16) & 1u;
  return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

float bf16_to_f32(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

float round_up_f32(double v) {
  float f = (float)v;
  if ((double)f < v) f = std::nextafter(f, INFINITY);
  return f;
}

// Error-bound constants of the refined path (see BoundCoef).  cmul is the
// vector the stored query values multiply (the codebook itself, or s*c for
// FP8 maps whose per-channel scale s is folded into the codebook); hi/lo are
// its BF16 split.  smax >= |s_d| bounds ||q|| by smax*||stored values||.
BoundCoef make_bound(const DeviceTemplate& t, const std::vector<double>& cmul,
                     const std::vector<float>& hi, const std::vector<float>& lo,
                     const std::vector<float>& cn32, bool f32_query, double smax) {
  const int D = t.D, k = t.k;
  const double u = 0x1.0p-23;  // per-addend relative error allowed to the accumulator
  const double n_add = (double)(f32_query ? 3 : 2) * t.geom.d_pad_bf16;
  const double gam = n_add * u / (1.0 - n_add * u);
  const double u64 = 0x1.0p-53;
  const double gam64 = (D + 2) * u64 / (1.0 - (D + 2) * u64);
  const double qfac = f32_query ? 1.0 + 0x1.0p-7 : 1.0;
  const double lofac = f32_query ? 0x1.0p-8 * (1.0 + 0x1.0p-7) : 0.0;
  const double rhofac = f32_query ? 0x1.0p-16 * (1.0 + 0x1.0p-6) : 0.0;
  const double pfac = f32_query ? (1.0 + 0x1.0p-7) * (1.0 + 0x1.0p-7) : 1.0;
  double A0 = 0.0, A1 = 0.0, cmax = 0.0;
  for (int j = 0; j < k; ++j) {
    double cn2 = 0.0, r2 = 0.0, a2 = 0.0, lo2 = 0.0;
    for (int d = 0; d < D; ++d) {
      double c = t.codebook[(size_t)j * D + d];
      double h = hi[(size_t)j * D + d], l = lo[(size_t)j * D + d];
      double r = cmul[(size_t)j * D + d] - h - l;   // exact: both sides fit 53 bits
      cn2 = cn2 + c * c;
      r2 = r2 + r * r;
      double a = std::fabs(h) + std::fabs(l);
      a2 = a2 + a * a;
      lo2 = lo2 + l * l;
    }
    const double slack = 1.0 + 0x1.0p-40;
    double cn = std::sqrt(cn2) * slack, rn = std::sqrt(r2) * slack;
    double an = std::sqrt(a2) * slack, lon = std::sqrt(lo2) * slack;
    double e_norm = std::fabs((double)cn32[j] - cn2) + (D + 2) * 0x1.0p-52 * cn2;
    // the products accumulate from zero (gamma bounds their rounding); the
    // FP32 norm is added once at the end (one more rounding of |s_j|)
    double a0j = e_norm + 0x1.0p-23 * std::fabs((double)cn32[j]);
    double a1j = 2.0 * (qfac * rn + lofac * lon + rhofac * cn) + 2.0 * gam * pfac * an +
                 0x1.0p-23 * 2.0 * (1.0 + 2.0 * gam) * pfac * an;
    A0 = std::max(A0, a0j);
    A1 = std::max(A1, a1j);
    cmax = std::max(cmax, cn);
  }
  // values below the normal range may be flushed by the matrix cores: an
  // absolute floor far above any such effect for finite inputs
  A0 += 1e-30;
  BoundCoef b;
  b.A0 = A0;
  b.A1 = A1;
  const double s = 1.0 + 0x1.0p-10;
  // 2*E64 with ||q|| <= smax*||e||: 2*gam64*(smax*||e|| + ||c||)^2
  b.a0 = round_up_f32(s * (2.0 * A0 + 2.0 * gam64 * cmax * cmax));
  b.a1 = round_up_f32(s * (2.0 * A1 + 4.0 * gam64 * cmax * smax));
  b.a2 = round_up_f32(s * (2.0 * gam64 * smax * smax));
  return b;
}

// BF16 hi/lo split of x (hi = x rounded to BF16 through FP32, lo = the rest
// rounded to BF16); the residual x - hi - lo is accounted for by make_bound.
void split_bf16(const std::vector<double>& x, std::vector<float>& hi, std::vector<float>& lo) {
  hi.resize(x.size());
  lo.resize(x.size());
  for (size_t i = 0; i < x.size(); ++i) {
    const float hf = bf16_to_f32(bf16_rne((float)x[i]));
    hi[i] = hf;
    lo[i] = bf16_to_f32(bf16_rne((float)(x[i] - (double)hf)));
  }
}

// MFMA A-operand fragments (-2 * hi, -2 * lo) in lane order.
void pack_frag_bf16(const DeviceTemplate& t, const std::vector<float>& hi, const std::vector<float>& lo,
                    std::vector<uint16_t>& out) {
  const int D = t.D, k = t.k;
  const AssignGeom& g = t.geom;
  const int S = g.s_bf16, KB = g.kb;
  const int steps = g.d_pad_bf16 / 32;
  out.assign((size_t)steps * 2 * KB * 64 * 8, 0);
  for (int st = 0; st < steps; ++st) {
    int gi = st / S, sp = st % S;
    for (int term = 0; term < 2; ++term)
      for (int mb = 0; mb < KB; ++mb)
        for (int l = 0; l < 64; ++l) {
          int m = l % 16, lg = l / 16;
          int j = 16 * mb + m;
          size_t base = ((((size_t)st * 2 + term) * KB + mb) * 64 + l) * 8;
          for (int i = 0; i < 8; ++i) {
            int d = 32 * S * gi + 8 * S * lg + 8 * sp + i;
            float v = 0.0f;
            if (j < k && d < D) v = -2.0f * (term == 0 ? hi : lo)[(size_t)j * D + d];
            out[base + i] = bf16_rne(v);
          }
        }
  }
}

// FP32 fragments (-2 * x) of the plain path in lane order.
void pack_frag_f32(const DeviceTemplate& t, const std::vector<float>& x, std::vector<float>& out) {
  const int D = t.D, k = t.k;
  const AssignGeom& g = t.geom;
  const int KB = g.kb, E = g.e_f32;
  const int fsteps = g.d_pad_f32 / 4;
  out.assign((size_t)fsteps * KB * 64, 0.0f);
  for (int st = 0; st < fsteps; ++st) {
    int gi = st / E, sp = st % E;
    for (int mb = 0; mb < KB; ++mb)
      for (int l = 0; l < 64; ++l) {
        int m = l % 16, lg = l / 16;
        int j = 16 * mb + m;
        int d = 4 * E * gi + E * lg + sp;
        float v = 0.0f;
        if (j < k && d < D) v = -2.0f * x[(size_t)j * D + d];
        out[((size_t)st * KB + mb) * 64 + l] = v;
      }
  }
}

}  // namespace

// Eigen-decomposition of a small symmetric matrix a [m][m] (row-major, FP64)
// by cyclic Jacobi rotations: on return the eigenvalues are on a's diagonal
// and v [m][m] holds the eigenvectors as columns.
static void jacobi_eigen(std::vector<double>& a, std::vector<double>& v, int m) {
  v.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) v[(size_t)i * m + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < m; ++i) {
      diag += a[(size_t)i * m + i] * a[(size_t)i * m + i];
      for (int j = i + 1; j < m; ++j) off += a[(size_t)i * m + j] * a[(size_t)i * m + j];
    }
    if (off <= 1e-30 * diag || off == 0.0) break;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = a[(size_t)p * m + q];
        if (apq == 0.0) continue;
        const double app = a[(size_t)p * m + p], aqq = a[(size_t)q * m + q];
        // rotation angle that zeroes a[p][q]: t = tan(theta), the smaller root
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < m; ++k) {           // columns p, q of a
          const double akp = a[(size_t)k * m + p], akq = a[(size_t)k * m + q];
          a[(size_t)k * m + p] = c * akp - sn * akq;
          a[(size_t)k * m + q] = sn * akp + c * akq;
        }
        for (int k = 0; k < m; ++k) {           // rows p, q of a
          const double apk = a[(size_t)p * m + k], aqk = a[(size_t)q * m + k];
          a[(size_t)p * m + k] = c * apk - sn * aqk;
          a[(size_t)q * m + k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < m; ++k) {           // eigenvector columns
          const double vkp = v[(size_t)k * m + p], vkq = v[(size_t)k * m + q];
          v[(size_t)k * m + p] = c * vkp - sn * vkq;
          v[(size_t)k * m + q] = sn * vkp + c * vkq;
        }
      }
  }
}

// Orthonormalises the m columns of q [D][m] (modified Gram-Schmidt, twice).
static void orthonormalise(std::vector<double>& q, int D, int m) {
  for (int pass = 0; pass < 2; ++pass)
    for (int j = 0; j < m; ++j) {
      for (int i = 0; i < j; ++i) {
        double dot = 0.0;
        for (int r = 0; r < D; ++r) dot += q[(size_t)r * m + i] * q[(size_t)r * m + j];
        for (int r = 0; r < D; ++r) q[(size_t)r * m + j] -= dot * q[(size_t)r * m + i];
      }
      double nrm = 0.0;
      for (int r = 0; r < D; ++r) nrm += q[(size_t)r * m + j] * q[(size_t)r * m + j];
      nrm = std::sqrt(nrm);
      for (int r = 0; r < D; ++r) q[(size_t)r * m + j] = nrm > 0 ? q[(size_t)r * m + j] / nrm : 0.0;
    }
}

void pca_fit_host(const float* x, int64_t n, int64_t stride, int D, int d, std::vector<double>& mean,
                  std::vector<double>& basis, std::vector<double>& var) {
  mean.assign(D, 0.0);
  for (int64_t p = 0; p < n; ++p)
    for (int t = 0; t < D; ++t) mean[t] = mean[t] + (double)x[p * stride + t];
  for (int t = 0; t < D; ++t) mean[t] = mean[t] / (double)n;
  std::vector<double> xc((size_t)n * D);
  for (int64_t p = 0; p < n; ++p)
    for (int t = 0; t < D; ++t) xc[(size_t)p * D + t] = (double)x[p * stride + t] - mean[t];
  // covariance, normalised by n; rows in parallel
  std::vector<double> cov((size_t)D * D, 0.0);
  parallel_for(D, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      double* ci = &cov[(size_t)i * D];
      for (int64_t p = 0; p < n; ++p) {
        const double xi = xc[(size_t)p * D + i];
        const double* xp = &xc[(size_t)p * D];
        for (int j = 0; j < D; ++j) ci[j] += xi * xp[j];
      }
      for (int j = 0; j < D; ++j) ci[j] /= (double)n;
    }
  }, 8);
  // subspace iteration with Rayleigh-Ritz on m >= d columns
  const int m = std::min(D, d + 8);
  std::vector<double> q((size_t)D * m), z((size_t)D * m), t((size_t)m * m), v, theta(m);
  uint64_t st = 0x243F6A8885A308D3ull;   // fixed start
  for (auto& e : q) {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t r = st;
    r = (r ^ (r >> 30)) * 0xBF58476D1CE4E5B9ull;
    r = (r ^ (r >> 27)) * 0x94D049BB133111EBull;
    e = (double)((r ^ (r >> 31)) >> 11) * 0x1.0p-53 - 0.5;
  }
  orthonormalise(q, D, m);
  auto mul_cov = [&](const std::vector<double>& in, std::vector<double>& out) {
    parallel_for(D, [&](int64_t b, int64_t e) {
      for (int64_t r = b; r < e; ++r)
        for (int j = 0; j < m; ++j) {
          double s2 = 0.0;
          for (int k = 0; k < D; ++k) s2 += cov[(size_t)r * D + k] * in[(size_t)k * m + j];
          out[(size_t)r * m + j] = s2;
        }
    }, 8);
  };
  for (int it = 0; it < 2000; ++it) {
    mul_cov(q, z);
    orthonormalise(z, D, m);
    // Rayleigh-Ritz: t = z^T C z, rotate z onto t's eigenvectors
    mul_cov(z, q);                                   // q <- C z
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        double s2 = 0.0;
        for (int r = 0; r < D; ++r) s2 += z[(size_t)r * m + i] * q[(size_t)r * m + j];
        t[(size_t)i * m + j] = s2;
      }
    for (int i = 0; i < m; ++i)
      for (int j = i + 1; j < m; ++j) {
        const double a2 = 0.5 * (t[(size_t)i * m + j] + t[(size_t)j * m + i]);
        t[(size_t)i * m + j] = t[(size_t)j * m + i] = a2;
      }
    jacobi_eigen(t, v, m);
    std::vector<int> order(m);
    for (int i = 0; i < m; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a2, int b2) { return t[(size_t)a2 * m + a2] > t[(size_t)b2 * m + b2]; });
    for (int r = 0; r < D; ++r)
      for (int j = 0; j < m; ++j) {
        double s2 = 0.0;
        for (int i = 0; i < m; ++i) s2 += z[(size_t)r * m + i] * v[(size_t)i * m + order[j]];
        q[(size_t)r * m + j] = s2;
      }
    for (int j = 0; j < m; ++j) theta[j] = t[(size_t)order[j] * m + order[j]];
    // converged when every wanted Ritz pair has a small residual
    if (it % 4 == 3 || it == 1999) {
      mul_cov(q, z);
      double worst = 0.0;
      for (int j = 0; j < d; ++j) {
        double r2 = 0.0;
        for (int r = 0; r < D; ++r) {
          const double e = z[(size_t)r * m + j] - theta[j] * q[(size_t)r * m + j];
          r2 += e * e;
        }
        worst = std::max(worst, std::sqrt(r2));
      }
      if (worst <= 1e-12 * std::max(theta[0], 1e-300)) break;
    }
  }
  basis.assign((size_t)d * D, 0.0);
  var.assign(d, 0.0);
  for (int j = 0; j < d; ++j) {
    int arg = 0;
    for (int r = 1; r < D; ++r)
      if (std::fabs(q[(size_t)r * m + j]) > std::fabs(q[(size_t)arg * m + j])) arg = r;
    const double sg = q[(size_t)arg * m + j] < 0 ? -1.0 : 1.0;
    for (int r = 0; r < D; ++r) basis[(size_t)j * D + r] = sg * q[(size_t)r * m + j];
    var[j] = theta[j];
  }
}

// Colour features of an RGB image: feature (3*dy + dx)*3 + c of pixel (x, y)
// is channel c of the pixel at (x + dx - 1, y + dy - 1), edges replicated.
void rgb_patch_features_host(const uint8_t* img, int H, int W, int64_t stride, float* out) {
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      float* f = out + ((size_t)y * W + x) * 27;
      for (int dy = 0; dy < 3; ++dy) {
        const int yy = std::min(std::max(y + dy - 1, 0), H - 1);
        for (int dx = 0; dx < 3; ++dx) {
          const int xx = std::min(std::max(x + dx - 1, 0), W - 1);
          const uint8_t* p = img + ((int64_t)yy * W + xx) * stride;
          for (int c = 0; c < 3; ++c) f[(3 * dy + dx) * 3 + c] = (float)p[c];
        }
      }
    }
}

// Builds every host table of a template from its FP32 codebook.
void prepare_template_host(DeviceTemplate& t, const float* tmpl, int64_t tmpl_stride,
                           const uint8_t* labels) {
  const int D = t.D, k = t.k;
  t.geom = make_assign_geom(k, D);
  int64_t n = (int64_t)t.w * t.h;
  if (labels) {
    t.labels.assign(labels, labels + n);
  } else {
    // template NNF with the exact FP64 rule
    std::vector<double> x((size_t)n * D), c((size_t)k * D);
    for (int64_t p = 0; p < n; ++p)
      for (int d = 0; d < D; ++d) x[(size_t)p * D + d] = (double)tmpl[p * tmpl_stride + d];
    for (size_t i = 0; i < c.size(); ++i) c[i] = (double)t.codebook[i];
    std::vector<int> lab = assign_host(x, n, D, c, k);
    t.labels.resize(n);
    for (int64_t p = 0; p < n; ++p) t.labels[p] = (uint8_t)lab[p];
  }
  // R(tau): per-filter counts over the template
  t.counts.clear();
  t.resp.clear();
  if (t.weighted) {
    // bin counts per group, then each filter's FP32 FMA chain over its
    // non-zero bins in row-major order (the bank kernel's order)
    t.resp.assign((size_t)t.n_filters * k, 0.0f);
    std::vector<float> cnt((size_t)16 * k);
    for (const BankGroup& g : t.groups) {
      std::fill(cnt.begin(), cnt.end(), 0.0f);
      for (int b = 0; b < g.gy; ++b)
        for (int a = 0; a < g.gx; ++a) {
          std::vector<int> hist(k, 0);
          for (int y = g.ye[b]; y < g.ye[b + 1]; ++y)
            for (int xx = g.xe[a]; xx < g.xe[a + 1]; ++xx) hist[t.labels[(size_t)y * t.w + xx]]++;
          for (int j = 0; j < k; ++j) cnt[(size_t)(b * 4 + a) * k + j] = (float)hist[j];
        }
      for (int f = g.f0; f < g.f1; ++f)
        for (int j = 0; j < k; ++j) {
          float r = 0.0f;
          for (int b = 0; b < g.gy; ++b)
            for (int a = 0; a < g.gx; ++a) {
              const float cv = t.coef[(size_t)f * 16 + b * 4 + a];
              if (cv != 0.0f) r = std::fmaf(cv, cnt[(size_t)(b * 4 + a) * k + j], r);
            }
          t.resp[(size_t)f * k + j] = r;
        }
    }
    return;
  }
  t.counts.assign((size_t)t.n_filters * k, 0);
  for (int f = 0; f < t.n_filters; ++f) {
    const int32_t* b = &t.boxes[(size_t)f * 4];
    for (int y = b[1]; y < b[3]; ++y)
      for (int xx = b[0]; xx < b[2]; ++xx) t.counts[(size_t)f * k + t.labels[(size_t)y * t.w + xx]]++;
  }
}

void build_tables(DeviceTemplate& t, HostTables& ht) {
  const int D = t.D, k = t.k;
  const AssignGeom& g = t.geom;
  std::vector<double> c64(t.codebook.begin(), t.codebook.end());
  std::vector<float> hi, lo;
  split_bf16(c64, hi, lo);
  // ||c||^2: FP64 sequential sum of squares, rounded to FP32
  ht.cnorm.assign(g.kpad, 3.0e38f);
  for (int j = 0; j < k; ++j) {
    double s = 0.0;
    for (int d = 0; d < D; ++d) {
      double v = t.codebook[(size_t)j * D + d];
      s = s + v * v;
    }
    ht.cnorm[j] = (float)s;
  }
  pack_frag_bf16(t, hi, lo, ht.frag_bf16);
  pack_frag_f32(t, t.codebook, ht.frag_f32);
  // counts (indicator banks) or responses (weighted banks) padded to kpad
  ht.resp.clear();
  if (t.weighted) {
    ht.resp.assign((size_t)t.n_filters * g.kpad, 0.0f);
    for (int f = 0; f < t.n_filters; ++f)
      for (int j = 0; j < k; ++j) ht.resp[(size_t)f * g.kpad + j] = t.resp[(size_t)f * k + j];
  }
  ht.counts.assign(t.weighted ? 0 : (size_t)t.n_filters * g.kpad, 0);
  ht.counts16.assign(t.weighted ? 0 : (size_t)t.n_filters * g.kpad / 2, 0);
  for (int f = 0; f < (t.weighted ? 0 : t.n_filters); ++f)
    for (int j = 0; j < k; ++j) {
      int32_t v = t.counts[(size_t)f * k + j];
      ht.counts[(size_t)f * g.kpad + j] = v;
      ht.counts16[(size_t)f * g.kpad / 2 + j / 2] |= ((uint32_t)v & 0xFFFFu) << (16 * (j & 1));
    }
  t.bound_bf16q = make_bound(t, c64, hi, lo, ht.cnorm, false, 1.0);
  t.bound_f32q = make_bound(t, c64, hi, lo, ht.cnorm, true, 1.0);
  t.cnorm32 = ht.cnorm;
}

// Tables for FP8 maps with per-channel scale s: the query codes e multiply
// c' = s*c (exact in FP64), split into BF16 hi/lo; q.c = e.c'.
void build_scaled_tables(const DeviceTemplate& t, const float* scale, std::vector<uint16_t>& frag_bf16,
                         std::vector<float>& frag_f32, BoundCoef& bound) {
  const int D = t.D, k = t.k;
  std::vector<double> cs((size_t)k * D);
  double smax = 0.0;
  for (int d = 0; d < D; ++d) smax = std::max(smax, std::fabs((double)scale[d]));
  for (int j = 0; j < k; ++j)
    for (int d = 0; d < D; ++d)
      cs[(size_t)j * D + d] = (double)scale[d] * (double)t.codebook[(size_t)j * D + d];
  std::vector<float> hi, lo, cs32(cs.size());
  split_bf16(cs, hi, lo);
  for (size_t i = 0; i < cs.size(); ++i) cs32[i] = (float)cs[i];
  pack_frag_bf16(t, hi, lo, frag_bf16);
  pack_frag_f32(t, cs32, frag_f32);
  bound = make_bound(t, cs, hi, lo, t.cnorm32, false, smax);
}

}  // namespace vqnnf
