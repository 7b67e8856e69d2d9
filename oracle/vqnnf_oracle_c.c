/*
 * FP64 CPU oracle for VQ-NNF template matching, C variant (Gupta & Sintorn,
 * arXiv 2306.15010).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check, the
 * benchmark's CPU-baseline leg and the scripts that write stored expected
 * values use it; the product path never does.  It shares no code, tables or
 * helpers with the GPU library.
 *
 * It computes the same quantities as the Python oracle (oracle/vqnnf_oracle.py),
 * in the same floating-point operations and the same order, so its results
 * are bit-identical to it (the CPU tests check that on every function);
 * it exists because the Python oracle cannot label the benchmark's
 * million-pixel maps in reasonable time.  Build with -ffp-contract=off and
 * without fast-math: every operation below is one correctly rounded IEEE
 * double operation.
 *
 *   O1  decode of stored elements: FP32, BF16 (the FP32 value whose upper
 *       16 bits are the pattern), OCP E4M3FN codes times a per-channel FP32
 *       scale (1 sign, 4 exponent bits with bias 7, 3 mantissa bits;
 *       exponent field 0 subnormal; no infinities).  Exact in double.
 *   O2  k-means of the template (Sec. 3.1, Sec. 4 "K-means computation",
 *       Sec. 5.2): seeded k-means++ with a splitmix64 stream, then Lloyd.
 *   O3  nearest-codeword assignment (Alg. 1, Sec. 3.1): squared L2 distance
 *       d = sum_t (q_t - c_t)^2 accumulated sequentially in t from 0 with a
 *       separate subtract, multiply and add; the lowest index wins ties.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define VQO_F32 0
#define VQO_BF16 1
#define VQO_FP8 2

/* ------------------------------------------------------------ O1 decode */

/* Value of one E4M3FN code from its fields (NaN for S.1111.111). */
double vqo_e4m3fn_value(int code) {
  const double sign = (code & 0x80) ? -1.0 : 1.0;
  const int e = (code >> 3) & 0xF, m = code & 7;
  if (e == 0xF && m == 7) return NAN;
  if (e == 0) return sign * ldexp((double)m, -9);        /* m/8 * 2^-6 */
  return sign * ldexp((double)(8 + m), e - 10);          /* (1 + m/8) * 2^(e-7) */
}

static double bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  memcpy(&f, &u, 4);
  return (double)f;
}

/* Decoded pixel p of a map (elements at q + p*stride) into out[D]. */
static void decode_pixel(const void* q, int dtype, int64_t p, int64_t stride, int D,
                         const float* scale, const double* e4m3, double* out) {
  if (dtype == VQO_F32) {
    const float* s = (const float*)q + p * stride;
    for (int t = 0; t < D; ++t) out[t] = (double)s[t];
  } else if (dtype == VQO_BF16) {
    const uint16_t* s = (const uint16_t*)q + p * stride;
    for (int t = 0; t < D; ++t) out[t] = bf16_value(s[t]);
  } else {
    const uint8_t* s = (const uint8_t*)q + p * stride;
    /* scale[d] * code value: a 24-bit times a 4-bit significand, exact */
    for (int t = 0; t < D; ++t) out[t] = e4m3[s[t]] * (double)scale[t];
  }
}

/* Decodes n pixels into out[n][D] (used by the tests to pin O1). */
int vqo_decode(const void* q, int dtype, int64_t n, int64_t stride, int D, const float* scale,
               double* out) {
  double e4m3[256];
  for (int c = 0; c < 256; ++c) e4m3[c] = vqo_e4m3fn_value(c);
  for (int64_t p = 0; p < n; ++p) decode_pixel(q, dtype, p, stride, D, scale, e4m3, out + p * D);
  return 0;
}

/* ------------------------------------------------------------ O3 assign */

/* acc[j] = sum_t (x[t] - ct[t][j])^2 for PB pixels at once (x: PB rows of
 * D), codebook transposed ct[D][k]; for each (pixel, j) the sum runs
 * sequentially in t (independent chains per j). */
static void distances_block(const double* x, int pb, int D, const double* ct, int k, double* acc) {
  for (int i = 0; i < pb * k; ++i) acc[i] = 0.0;
  for (int t = 0; t < D; ++t) {
    const double* row = ct + (int64_t)t * k;
    for (int b = 0; b < pb; ++b) {
      const double xt = x[(int64_t)b * D + t];
      double* a = acc + (int64_t)b * k;
      for (int j = 0; j < k; ++j) {
        const double diff = xt - row[j];
        const double sq = diff * diff;
        a[j] = a[j] + sq;
      }
    }
  }
}

typedef struct {
  const void* q;
  int dtype;
  int64_t p0, p1, stride;
  int D, k;
  const float* scale;
  const double* ct;
  const double* e4m3;
  uint8_t* labels;     /* or NULL */
  double* dist;        /* [n][k] or NULL */
  int rc;
} AssignJob;

#define PB 4

static void* assign_worker(void* arg) {
  AssignJob* j = (AssignJob*)arg;
  const int D = j->D, k = j->k;
  double* x = (double*)malloc(sizeof(double) * PB * D);
  double* acc = (double*)malloc(sizeof(double) * PB * k);
  if (!x || !acc) {
    free(x);
    free(acc);
    j->rc = -1;
    return NULL;
  }
  for (int64_t p = j->p0; p < j->p1; p += PB) {
    const int pb = (int)((j->p1 - p) < PB ? (j->p1 - p) : PB);
    for (int b = 0; b < pb; ++b) decode_pixel(j->q, j->dtype, p + b, j->stride, D, j->scale, j->e4m3, x + (int64_t)b * D);
    distances_block(x, pb, D, j->ct, k, acc);
    for (int b = 0; b < pb; ++b) {
      const double* a = acc + (int64_t)b * k;
      if (j->dist) memcpy(j->dist + (p + b) * (int64_t)k, a, sizeof(double) * k);
      if (j->labels) {
        int best = 0;
        for (int c = 1; c < k; ++c)
          if (a[c] < a[best]) best = c;   /* strict: the first minimum wins */
        j->labels[p + b] = (uint8_t)best;
      }
    }
  }
  free(x);
  free(acc);
  j->rc = 0;
  return NULL;
}

/* Labels (uint8, k <= 256) and/or FP64 distances [n][k] of n pixels of a
 * stored map against an FP64 codebook [k][D], on n_threads threads (the
 * result does not depend on the thread count). */
int vqo_assign(const void* q, int dtype, int64_t n, int64_t stride, int D, const float* scale,
               const double* codebook, int k, uint8_t* labels, double* dist, int n_threads) {
  if (k < 1 || k > 256 || D < 1 || n < 0) return -2;
  double e4m3[256];
  for (int c = 0; c < 256; ++c) e4m3[c] = vqo_e4m3fn_value(c);
  double* ct = (double*)malloc(sizeof(double) * (size_t)k * D);
  if (!ct) return -1;
  for (int j = 0; j < k; ++j)
    for (int t = 0; t < D; ++t) ct[(int64_t)t * k + j] = codebook[(int64_t)j * D + t];
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 256) n_threads = 256;
  AssignJob jobs[256];
  pthread_t th[256];
  const int64_t per = (n + n_threads - 1) / n_threads;
  int started = 0, rc = 0;
  for (int i = 0; i < n_threads; ++i) {
    AssignJob* j = &jobs[i];
    j->q = q; j->dtype = dtype; j->stride = stride; j->D = D; j->k = k; j->scale = scale;
    j->ct = ct; j->e4m3 = e4m3; j->labels = labels; j->dist = dist; j->rc = 0;
    j->p0 = (int64_t)i * per < n ? (int64_t)i * per : n;
    j->p1 = j->p0 + per < n ? j->p0 + per : n;
    if (n_threads == 1) {
      assign_worker(j);
      started = 0;
      rc = j->rc;
      break;
    }
    if (pthread_create(&th[i], NULL, assign_worker, j) != 0) { rc = -1; break; }
    ++started;
  }
  for (int i = 0; i < started; ++i) {
    pthread_join(th[i], NULL);
    if (jobs[i].rc) rc = jobs[i].rc;
  }
  free(ct);
  return rc;
}

/* ------------------------------------------------------------ O2 k-means */

/* Vigna's splitmix64; u01 = (next >> 11) * 2^-53. */
static uint64_t sm_next(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static double sm_u01(uint64_t* s) { return (double)(sm_next(s) >> 11) * 0x1.0p-53; }

/* First outputs of the generator (pinned by the tests against published values). */
void vqo_splitmix64(uint64_t seed, int n, uint64_t* out, double* u) {
  uint64_t s = seed;
  for (int i = 0; i < n; ++i) out[i] = sm_next(&s);
  s = seed;
  for (int i = 0; i < n; ++i) u[i] = sm_u01(&s);
}

static int64_t uniform_index(double u, int64_t n) {
  const int64_t i = (int64_t)floor(u * (double)n);
  return i < n - 1 ? i : n - 1;
}

/* squared distance of point x[D] to centre c[D], sequential in t */
static double sqd(const double* x, const double* c, int D) {
  double acc = 0.0;
  for (int t = 0; t < D; ++t) {
    const double diff = x[t] - c[t];
    const double sq = diff * diff;
    acc = acc + sq;
  }
  return acc;
}

typedef struct {
  const double* x;
  const double* ct;
  int64_t p0, p1;
  int D, k;
  int* lab;
  int rc;
} LloydJob;

static void* lloyd_worker(void* arg) {
  LloydJob* j = (LloydJob*)arg;
  double* acc = (double*)malloc(sizeof(double) * PB * j->k);
  if (!acc) { j->rc = -1; return NULL; }
  for (int64_t p = j->p0; p < j->p1; p += PB) {
    const int pb = (int)((j->p1 - p) < PB ? (j->p1 - p) : PB);
    distances_block(j->x + p * j->D, pb, j->D, j->ct, j->k, acc);
    for (int b = 0; b < pb; ++b) {
      const double* a = acc + (int64_t)b * j->k;
      int best = 0;
      for (int c = 1; c < j->k; ++c)
        if (a[c] < a[best]) best = c;
      j->lab[p + b] = best;
    }
  }
  free(acc);
  j->rc = 0;
  return NULL;
}

/* Nearest centre of every point (first minimum), on n_threads threads. */
static int nearest(const double* x, int64_t l, int D, const double* c, int k, int* lab, int n_threads) {
  double* ct = (double*)malloc(sizeof(double) * (size_t)k * D);
  if (!ct) return -1;
  for (int j = 0; j < k; ++j)
    for (int t = 0; t < D; ++t) ct[(int64_t)t * k + j] = c[(int64_t)j * D + t];
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 256) n_threads = 256;
  LloydJob jobs[256];
  pthread_t th[256];
  const int64_t per = (l + n_threads - 1) / n_threads;
  int started = 0, rc = 0;
  for (int i = 0; i < n_threads; ++i) {
    LloydJob* j = &jobs[i];
    j->x = x; j->ct = ct; j->D = D; j->k = k; j->lab = lab; j->rc = 0;
    j->p0 = (int64_t)i * per < l ? (int64_t)i * per : l;
    j->p1 = j->p0 + per < l ? j->p0 + per : l;
    if (n_threads == 1) {
      lloyd_worker(j);
      rc = j->rc;
      break;
    }
    if (pthread_create(&th[i], NULL, lloyd_worker, j) != 0) { rc = -1; break; }
    ++started;
  }
  for (int i = 0; i < started; ++i) {
    pthread_join(th[i], NULL);
    if (jobs[i].rc) rc = jobs[i].rc;
  }
  free(ct);
  return rc;
}

/* k-means codebook of l points (FP32 rows [l][D], row-major template order):
 *  k-means++: the first centre is point floor(u*l) (clamped) for u = u01();
 *  D^2 is every point's squared distance to its nearest chosen centre; each
 *  next centre takes u = u01() and is the first point whose sequential
 *  running sum of D^2 exceeds u * S, S the sequential total (the last point
 *  with a positive D^2 if none does), or a uniform draw floor(u*l) when
 *  S == 0; after each draw D^2 = min(D^2, distance to the new centre).
 *  Lloyd, `iters` times: every point to its nearest centre (first minimum),
 *  then every non-empty cluster's centre = (sequential FP64 sum of its points
 *  in point order) / count; an empty cluster keeps its centre.
 * out64: [k][D] FP64 centres; out32: the same rounded to FP32 (either may be
 * NULL). */
int vqo_kmeans(const float* pts, int64_t l, int D, int k, int iters, uint64_t seed, double* out64,
               float* out32, int n_threads) {
  if (l < 1 || D < 1 || k < 1 || iters < 0) return -2;
  double* x = (double*)malloc(sizeof(double) * (size_t)l * D);
  double* c = (double*)malloc(sizeof(double) * (size_t)k * D);
  double* d2 = (double*)malloc(sizeof(double) * (size_t)l);
  int* lab = (int*)malloc(sizeof(int) * (size_t)l);
  double* s = (double*)malloc(sizeof(double) * (size_t)D);
  int rc = 0;
  if (!x || !c || !d2 || !lab || !s) { rc = -1; goto done; }
  for (int64_t i = 0; i < l * (int64_t)D; ++i) x[i] = (double)pts[i];
  uint64_t st = seed;
  /* k-means++ */
  {
    const int64_t first = uniform_index(sm_u01(&st), l);
    memcpy(c, x + first * D, sizeof(double) * D);
    for (int64_t p = 0; p < l; ++p) d2[p] = sqd(x + p * D, c, D);
    for (int i = 1; i < k; ++i) {
      /* running sums start at the first term (d2 >= +0, so 0.0 + d2[0] would
         be the same value) */
      double total = d2[0];
      for (int64_t p = 1; p < l; ++p) total = total + d2[p];
      const double u = sm_u01(&st);
      int64_t idx;
      if (total == 0.0) {
        idx = uniform_index(u, l);
      } else {
        const double target = u * total;
        double run = 0.0;
        idx = -1;
        for (int64_t p = 0; p < l; ++p) {
          run = p == 0 ? d2[0] : run + d2[p];
          if (run > target) { idx = p; break; }
        }
        if (idx < 0) {
          for (int64_t p = l - 1; p >= 0; --p)
            if (d2[p] > 0.0) { idx = p; break; }
        }
      }
      memcpy(c + (int64_t)i * D, x + idx * D, sizeof(double) * D);
      for (int64_t p = 0; p < l; ++p) {
        const double dn = sqd(x + p * D, c + (int64_t)i * D, D);
        if (dn < d2[p]) d2[p] = dn;
      }
    }
  }
  /* Lloyd */
  for (int it = 0; it < iters; ++it) {
    if ((rc = nearest(x, l, D, c, k, lab, n_threads))) goto done;
    for (int j = 0; j < k; ++j) {
      int64_t cnt = 0;
      for (int64_t p = 0; p < l; ++p) {
        if (lab[p] != j) continue;
        const double* xp = x + p * D;
        if (cnt == 0)   /* the running sum starts at the first point itself */
          for (int t = 0; t < D; ++t) s[t] = xp[t];
        else
          for (int t = 0; t < D; ++t) s[t] = s[t] + xp[t];
        ++cnt;
      }
      if (cnt == 0) continue;
      for (int t = 0; t < D; ++t) c[(int64_t)j * D + t] = s[t] / (double)cnt;
    }
  }
  if (out64) memcpy(out64, c, sizeof(double) * (size_t)k * D);
  if (out32)
    for (int64_t i = 0; i < (int64_t)k * D; ++i) out32[i] = (float)c[i];
done:
  free(x);
  free(c);
  free(d2);
  free(lab);
  free(s);
  return rc;
}
