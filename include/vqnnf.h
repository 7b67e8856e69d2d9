/*
 * vqnnf.h - C ABI of the MI355X (gfx950) VQ-NNF template-matching library.
 *
 * The library implements the data-parallel hot path of
 *   Gupta & Sintorn, "Efficient High-Resolution Template Matching with Vector
 *   Quantized Nearest Neighbour Fields" (arXiv 2306.15010):
 *     codebook + NNF creation (Sec. 3.1, Alg. 1), one-hot integral images
 *     (Sec. 3.1, Supp. S.2), coarse filters on integral images (Sec. 3.2,
 *     eq. 1, Alg. 2), similarity (Sec. 3.3, eq. 2), localisation (Sec. 4).
 *
 * Problem statement (Sec. 3): a template tau of w x h x c and a query I of
 * W x H x c; a similarity score for every w x h sub-window of I, and the best
 * one.  Here c is called D (feature dimension).
 *
 * Conventions shared by every call:
 *  - Feature maps are HWC: element (y, x, d) of a map sits at
 *    data[(y*W + x)*pixel_stride + d], pixel_stride >= D elements.
 *  - Pointers documented as "device" are HIP device pointers (e.g. a torch
 *    tensor's data_ptr()); "host" pointers are ordinary CPU memory.
 *  - The caller owns every input and output buffer.  The library owns its
 *    handles and its scratch memory (capped by scratch_cap_bytes).
 *  - Every GPU call is enqueued on the context's HIP stream and returns
 *    before the work completes, except where a host output (best location,
 *    flagged count) is requested: those calls synchronise the stream.
 *  - Argument validation happens before any HIP call.  On error the call
 *    returns a non-zero status, leaves no work enqueued, and
 *    vqnnf_last_error() describes the problem (thread-local string).  Output
 *    buffers are unspecified after an error.
 *  - All floating-point inputs must be finite.
 */
#ifndef VQNNF_H
#define VQNNF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VQNNF_OK = 0,
  VQNNF_EINVAL = 1,   /* invalid argument (null pointer, bad size, bad enum) */
  VQNNF_ENOMEM = 2,   /* scratch cap exceeded or device allocation failed   */
  VQNNF_EHIP = 3,     /* a HIP runtime call failed                          */
  VQNNF_ENOTSUP = 4,  /* device is not gfx950, or combination not supported  */
  VQNNF_EHANDLE = 5   /* null or already-freed handle                       */
} vqnnf_status;

/* Storage type of a feature map. */
typedef enum {
  VQNNF_F32 = 0,      /* IEEE binary32                                      */
  VQNNF_BF16 = 1,     /* bfloat16 bit patterns (uint16)                     */
  VQNNF_FP8_E4M3 = 2, /* OCP E4M3FN codes (uint8) times a per-channel scale */
  /* uint8 RGB image whose features are its colour patches (Sec. 5.2
   * "Feature Extraction"): D = 27, feature (3*dy + dx)*3 + c of pixel (x, y)
   * is channel c of the pixel at (x + dx - 1, y + dy - 1), dx, dy in 0..2,
   * neighbours outside the image replaced by the nearest pixel inside, values
   * 0..255.  pixel_stride counts bytes (>= 3; 0 means 3). */
  VQNNF_RGB8 = 3
} vqnnf_dtype;

/* Arithmetic used for the nearest-codeword search. */
typedef enum {
  /* FP32 matrix-core distances ||c||^2 - 2 q.c and a plain argmin.  No
   * refinement: a label may differ from the exact FP64 nearest neighbour
   * when two codewords are nearly equidistant. */
  VQNNF_PREC_FP32_PLAIN = 0,
  /* BF16 matrix-core distances with FP32 accumulation (codebook split into
   * BF16 hi + lo terms; FP32-stored queries split too), a per-pixel error
   * bound, and an FP64 re-score of every pixel whose best-to-second gap is
   * inside the bound.  Labels equal the FP64 nearest neighbour computed in
   * the fixed order d = sum_t (q_t - c_t)^2 (sequential in t, no FMA),
   * lowest index on ties. */
  VQNNF_PREC_BF16_REFINED = 1,
  /* For VQNNF_FP8_E4M3 maps only (else VQNNF_EINVAL): the same refined
   * search as VQNNF_PREC_BF16_REFINED, which FP8 maps take anyway (the E4M3
   * codes are exact in BF16, the channel scale is folded into a copy of the
   * codebook); the FP64 re-score uses code x scale, the oracle's value. */
  VQNNF_PREC_FP8_REFINED = 2
} vqnnf_prec;

/* A feature map (query or template). */
typedef struct {
  const void* data;            /* see each call for host/device            */
  int32_t dtype;               /* vqnnf_dtype                               */
  int32_t H, W, D;             /* rows, columns, feature dimension          */
  int64_t pixel_stride;        /* elements between pixels; 0 means D; one
                                  pixel row is at most 4 MiB (else EINVAL) */
  const float* channel_scale;  /* FP8 only: host float[D]; else NULL        */
} vqnnf_fmap;

/* One entry of the filter bank (Sec. 3.2): the region [x0,x1) x [y0,y1) of
 * the template, split into a gx x gy grid with bin edges
 * x0 + floor(a*(x1-x0)/gx), y0 + floor(b*(y1-y0)/gy).
 *  - bin_weight == NULL: every bin is its own indicator filter (a k-channel
 *    histogram); its score weight is weight / (gx*gy*area(bin)).
 *  - bin_weight != NULL: one coarse filter (Sec. 3.2.1, eq. 1 with Alg. 2's
 *    dilation taps on the bin corners): its response on channel j is
 *    sum_{b,a} bin_weight[b*gx + a] * count_j(bin (a, b)) / area(region),
 *    scored with weight `weight`.  gx and gy are at most 4 (else
 *    VQNNF_ENOTSUP) and every bin weight must be finite; the array is read
 *    during the call only.  Such banks are scored from the integral image. */
typedef struct {
  int32_t x0, y0, x1, y1;
  int32_t gx, gy;
  const float* bin_weight;     /* host, gy*gx row-major, or NULL            */
  float weight;
} vqnnf_filter_desc;

typedef struct vqnnf_ctx vqnnf_ctx;
typedef struct vqnnf_template vqnnf_template;

/* The paper's filter sets (Sec. 5.2 "Filtering"): a 3x3 coarse Gaussian
 * (sigma 2, unnormalised: exp(-(a^2 + b^2)/8) for a, b in {-1, 0, 1}) alone
 * or with Haar-like filters multiplied by it elementwise: 2-rectangle x / y
 * (column / row factors +1, 0, -1) and 3-rectangle x / y (+1, -2, +1). */
typedef enum {
  VQNNF_BANK_GAUSS = 0,    /* Gaussian                       (1 per scale) */
  VQNNF_BANK_2RECT = 1,    /* Gaussian, Haar-2x, Haar-2y     (3 per scale) */
  VQNNF_BANK_3RECT = 2,    /* Gaussian, Haar-3x, Haar-3y     (3 per scale) */
  VQNNF_BANK_23RECT = 3    /* Gaussian, 2x, 2y, 3x, 3y       (5 per scale) */
} vqnnf_bank_set;

/* Fills the paper's bank for a w x h template (Sec. 3.2.2, Sec. 3.3 eq. 2,
 * Sec. 5.2; sub-scale aggregation is Supp. S.3's option c).  For every scale
 * s = 1..n_scales: the centred sub-window of floor(w/s) x floor(h/s) pixels
 * starting at (floor((w - floor(w/s))/2), floor((h - floor(h/s))/2)), a 3x3
 * grid, one weighted filter per member of the set, weight w_f / s with
 * w_f = 1 for the Gaussian and 0.25 for the Haar filters.  Order: scale by
 * scale, within a scale Gaussian, 2x, 2y, 3x, 3y (members of the set only).
 *  out: HOST array of `capacity` descs; bin_weights: HOST float[9*capacity];
 *  desc i's bin_weight points at bin_weights + 9*i, so that array must stay
 *  alive while the descs are used.  n_out: descs written.
 * EINVAL (nothing written) for an unknown set, n_scales < 1, capacity below
 * n_scales * set size, null pointers, or a sub-window under 3 x 3 pixels.
 * Host only; needs no context. */
vqnnf_status vqnnf_paper_bank(int32_t w, int32_t h, int32_t filter_set, int32_t n_scales,
                              vqnnf_filter_desc* out, float* bin_weights, int32_t capacity,
                              int32_t* n_out);

/* Creates a context bound to the current HIP device and `hip_stream`
 * (a hipStream_t; NULL = the default stream).  scratch_cap_bytes bounds the
 * device scratch the context may hold (0 = 16 GiB).  Returns ENOTSUP if the
 * current device is not gfx950. */
vqnnf_status vqnnf_ctx_create(void* hip_stream, uint64_t scratch_cap_bytes, vqnnf_ctx** out);

/* Creates a context with no device.  Templates are prepared on the host
 * (k-means, template NNF, counts and every getter work); every GPU call
 * validates its arguments and the scratch cap, then returns VQNNF_ENOTSUP.
 * Useful for host-only tools and for checking argument handling. */
vqnnf_status vqnnf_ctx_create_host(uint64_t scratch_cap_bytes, vqnnf_ctx** out);
void vqnnf_ctx_destroy(vqnnf_ctx* ctx);

/* Template preparation (Sec. 3.1, Sec. 4 "K-means computation"): k-means of
 * the template's w*h feature vectors (row-major order), seeded k-means++
 * (splitmix64 stream from `seed`) then exactly `lloyd_iters` Lloyd
 * iterations in FP64, rounded to FP32; then the template's NNF (same FP64
 * rule as VQNNF_PREC_BF16_REFINED) and its representation R(tau): the
 * counts of every filter of `bank` over the template (Sec. 3.3).
 *  tmpl: HOST map, dtype VQNNF_F32, H = h, W = w.
 *  k in [1, 256]; bank: host array of n_desc >= 1 entries, each region
 *  inside [0,w) x [0,h) with non-empty bins.
 * On a device context the k-means and the template NNF run on the GPU
 * (FP64, the same operations in the same order, so the result is bit-identical
 * to the host definition); on a host context they run on the host.  The
 * handle's tables are uploaded to the device. */
vqnnf_status vqnnf_codebook(vqnnf_ctx* ctx, const vqnnf_fmap* tmpl, int32_t k, int32_t lloyd_iters,
                            uint64_t seed, const vqnnf_filter_desc* bank, int32_t n_desc,
                            vqnnf_template** out);

/* vqnnf_codebook for n templates at once: template i has map tmpls[i],
 * k = ks[i], seed seeds[i] and bank banks[i] (n_descs[i] entries); every
 * template runs lloyd_iters iterations.  On a device context the k-means of
 * all templates (and their NNFs) run on the GPU together, bit-identical to
 * the host definition above; on a host context they run on the host.  out:
 * n handles, all NULL on error (EINVAL names the template).  Temporary device
 * memory is allocated and released inside the call (within the scratch cap). */
vqnnf_status vqnnf_codebook_batched(vqnnf_ctx* ctx, int32_t n, const vqnnf_fmap* const* tmpls,
                                    const int32_t* ks, int32_t lloyd_iters, const uint64_t* seeds,
                                    const vqnnf_filter_desc* const* banks, const int32_t* n_descs,
                                    vqnnf_template** out);

/* Dimensionality reduction (Sec. 5.5): PCA of the template's features, the
 * pixels mean-centred, covariance normalised by the pixel count (FP64), the d
 * axes of largest variance in decreasing order, each with its
 * largest-magnitude component positive.
 *  tmpl: HOST map (F32, or RGB8 for colour features), as for vqnnf_codebook.
 *  d in [1, min(D, 64)].  mean: HOST float[D]; basis: HOST float[d][D] (row i
 *  is axis i); variances: HOST float[d] or NULL.  Host only; EINVAL on bad
 *  arguments. */
vqnnf_status vqnnf_pca_fit(const vqnnf_fmap* tmpl, int32_t d, float* mean, float* basis, float* variances);

/* Projects a DEVICE map onto d axes: out[(y*W + x)*d + i] =
 * sum_t (q_t - mean_t) * basis[i][t] for every pixel, where q_t is the map's
 * element value (FP8: code x scale rounded to FP32; RGB8: colour feature t).
 * Arithmetic: FP32, the subtraction rounded and the products accumulated by
 * FMA in increasing t; BF16 maps with D a multiple of 32 and 16-byte aligned
 * rows use the matrix cores instead: exact products of the elements with an
 * exact three-term BF16 split of the basis, FP32 accumulation, then minus
 * mean . basis (computed in FP64, rounded once).  mean/basis: HOST, as from vqnnf_pca_fit; out: DEVICE
 * float[H*W*d].  The result is an F32 map of D = d for vqnnf_codebook (after
 * copying a projected template back) and every matching call.  Asynchronous
 * on the context stream. */
vqnnf_status vqnnf_pca_project(vqnnf_ctx* ctx, const vqnnf_fmap* map, const float* mean,
                               const float* basis, int32_t d, float* out);

/* Same as vqnnf_codebook but with a caller-supplied codebook (host float
 * [k][D], FP32) instead of k-means: used to restore an exported template and
 * to run every stage against an independently computed codebook. */
vqnnf_status vqnnf_template_from_codebook(vqnnf_ctx* ctx, const vqnnf_fmap* tmpl,
                                          const float* codebook, int32_t k,
                                          const vqnnf_filter_desc* bank, int32_t n_desc,
                                          vqnnf_template** out);
void vqnnf_template_free(vqnnf_template* t);

/* Template getters (host outputs).  info: w, h, D, k, number of expanded
 * filters.  codebook: float[k][D].  labels: uint8[h][w].  counts: int32
 * [n_filters][k] (R(tau)).  weights: float[n_filters]. */
vqnnf_status vqnnf_template_info(const vqnnf_template* t, int32_t* w, int32_t* h, int32_t* D,
                                 int32_t* k, int32_t* n_filters);
vqnnf_status vqnnf_template_codebook(const vqnnf_template* t, float* out);
vqnnf_status vqnnf_template_labels(const vqnnf_template* t, uint8_t* out);
vqnnf_status vqnnf_template_counts(const vqnnf_template* t, int32_t* out);
vqnnf_status vqnnf_template_weights(const vqnnf_template* t, float* out);
/* R(tau) as the score kernels read it: float[n_filters][k], each filter's
 * FP32 response over the template (an indicator filter: its counts; a
 * weighted filter: the FMA chain over its non-zero bins in row-major order,
 * coefficient bin_weight / area(region) rounded to FP32).  Works for every
 * bank; vqnnf_template_counts returns VQNNF_ENOTSUP for banks with weighted
 * filters. */
vqnnf_status vqnnf_template_responses(const vqnnf_template* t, float* out);

/* NNF of a query map (Alg. 1): labels[y*W + x] = index of the nearest
 * codeword of pixel (y, x) (squared L2, lowest index on ties).
 *  query: DEVICE map, dtype F32, BF16, FP8_E4M3 (with its host channel
 *  scales) or RGB8 (D = 27 colour features), query->D == template D.
 *  prec: a vqnnf_prec (VQNNF_PREC_FP8_REFINED with FP8 maps only).
 *  labels: DEVICE uint8[H*W].
 *  n_flagged: HOST, may be NULL; receives the number of pixels re-scored in
 *  FP64 (0 for VQNNF_PREC_FP32_PLAIN).  Non-NULL synchronises. */
vqnnf_status vqnnf_assign(vqnnf_ctx* ctx, const vqnnf_template* t, const vqnnf_fmap* query,
                          int32_t prec, uint8_t* labels, int64_t* n_flagged);

/* One-hot integral image of a label map (Sec. 3.1, Supp. S.2):
 *   integral[(y*(W+1) + x)*k + j] = #{(x', y') : y' < y, x' < x,
 *                                      labels[y'*W + x'] == j}
 * for 0 <= y <= H, 0 <= x <= W (exclusive and zero padded, channel-last,
 * exact int32; the paper's inclusive value at (x, y) is entry (y+1, x+1)).
 *  labels: DEVICE uint8[H*W], every value < k.  integral: DEVICE int32
 *  [(H+1)*(W+1)*k].  Requires (H+1)*(W+1)*k < 2^62 and H*W < 2^31. */
vqnnf_status vqnnf_filter(vqnnf_ctx* ctx, const vqnnf_template* t, const uint8_t* labels,
                          int32_t H, int32_t W, int32_t* integral);

/* Similarity heatmap from a label map (Sec. 3.2-3.3, eq. 2, Sec. 4):
 *   heatmap[y*(W-w+1) + x] = -sum_f weight_f * sum_j |R_f,j(tau) - C_f,j(x,y)|
 * where C_f,j(x,y) counts label j in filter f's box shifted to the window
 * whose top-left is (x, y); only windows inside the map are scored.  The
 * per-filter L1 is exact integer arithmetic, and so is its sum over the
 * bins of one weight; the weighted sum is FP32: the full window, then one
 * term per distinct bin weight in order of first appearance.
 * best_xy/best_score: HOST, may be NULL; the first maximum in row-major
 * order (non-NULL synchronises).
 *  labels: DEVICE uint8[H*W]; heatmap: DEVICE float[(H-h+1)*(W-w+1)];
 *  requires w <= W, h <= H.  VQNNF_ENOTSUP for banks other than the full
 *  window + g x g grid (g <= 4) with at most four distinct bin weights, or
 *  beyond the on-chip tile's width; vqnnf_filter + vqnnf_score_integral
 *  take those. */
vqnnf_status vqnnf_score(vqnnf_ctx* ctx, const vqnnf_template* t, const uint8_t* labels,
                         int32_t H, int32_t W, float* heatmap, int32_t* best_xy,
                         float* best_score);

/* Same heatmap computed from a one-hot integral image produced by
 * vqnnf_filter (the taps of Alg. 2's dilation filters read directly from
 * `integral`, DEVICE int32[(H+1)*(W+1)*k]), for any bank.  With weighted
 * filters, R_f,j(x,y) is the filter's response (bin counts exact in
 * integers, then the FP32 FMA chain of vqnnf_template_responses) and the
 * L1 over channels and the weighted sum are FP32. */
vqnnf_status vqnnf_score_integral(vqnnf_ctx* ctx, const vqnnf_template* t,
                                  const int32_t* integral, int32_t H, int32_t W, float* heatmap,
                                  int32_t* best_xy, float* best_score);

/* The whole hot path for one (template, query) pair: vqnnf_assign, then the
 * filter bank and eq. 2 on the resulting NNF (integral images built tile by
 * tile on chip), then localisation.  Arguments as in vqnnf_assign and
 * vqnnf_score; the label map lives in library scratch. */
vqnnf_status vqnnf_match(vqnnf_ctx* ctx, const vqnnf_template* t, const vqnnf_fmap* query,
                         int32_t prec, float* heatmap, int32_t* best_xy, float* best_score);

/* vqnnf_match for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments and the same results as vqnnf_match, bit for bit, with
 * every intermediate (label map, re-score worklist and candidate masks,
 * score partial sums, best-location key) placed in one fixed device array
 * of VQNNF_NOALLOC_SCRATCH_BYTES that the library holds on each device it
 * runs on until the process ends.  The call allocates nothing (no hipMalloc,
 * hipFree or event creation) and does not autotune (it uses the score tile
 * choice tuned by an earlier vqnnf_match on the same shape, else the
 * default) or record kernel timings.
 *  - VQNNF_ENOMEM when the pair needs more than the array holds: about
 *    H*W*(1 + 4 + 4*ceil(k/32)) bytes on the refined path (H*W on the plain
 *    path) plus the score's partial sums, e.g. a 1024 x 1024 map with k = 128
 *    and a 96 x 96 template takes 35 MB.
 *  - VQNNF_ENOTSUP for banks the on-chip score does not take (see
 *    vqnnf_score).
 *  - FP8 maps: EINVAL unless the template already holds the codebook tables
 *    of the map's channel scales (built by any vqnnf_assign, vqnnf_match or
 *    vqnnf_match_batched call with a map of the same scales).
 * Every call on one device shares that device's array, which keeps the last
 * call's contents (each call clears what must start at zero): calls whose
 * work overlaps on one device (different streams or contexts, host threads)
 * race and give wrong results; serialise them. */
#define VQNNF_NOALLOC_SCRATCH_BYTES ((uint64_t)64 << 20)
vqnnf_status vqnnf_match_noalloc(vqnnf_ctx* ctx, const vqnnf_template* t, const vqnnf_fmap* query,
                                 int32_t prec, float* heatmap, int32_t* best_xy, float* best_score);

/* A batch of independent (template, query map) pairs, the whole path for
 * each: t[i] is matched against q[i] into heatmaps[i] (device,
 * (H_i - h_i + 1) x (W_i - w_i + 1) FP32, caller owned), with the same
 * precision for every pair.  Templates and maps may differ in size, k, D
 * and storage, and the same map may appear in several pairs.  best_xy
 * (host, 2*n_pairs) and best_score (host, n_pairs) receive each pair's
 * localisation (Sec. 4); both NULL skips the synchronisation.  Every pair
 * is validated before anything is enqueued (EINVAL names the pair).
 * Launch structure (BF16-refined, BF16/FP8 maps): one fused assignment
 * launch per (storage, D) class that assigns every map of the class against
 * all of its templates, then for the whole batch one FP64 re-score launch,
 * one score launch per grid size and one combine launch per stored-sum
 * count, each reading its pairs' arguments from a device table; other pairs
 * run the single-pair path in turn.  Results equal
 * vqnnf_match's for every pair, bit for bit.  With
 * graph mode on (vqnnf_ctx_set_graph) the batch's kernels are captured into
 * one HIP graph and later calls with the same arguments (handles, pointers,
 * sizes, precision) replay it as a single launch; the inputs' contents may
 * change between calls, the handles and buffers must stay alive. */
vqnnf_status vqnnf_match_batched(vqnnf_ctx* ctx, int32_t n_pairs, const vqnnf_template* const* t,
                                 const vqnnf_fmap* const* q, int32_t prec, float* const* heatmaps,
                                 int32_t* best_xy, float* best_score);

/* The NNF label map (Alg. 1) that the last vqnnf_match_batched call on this
 * context computed for pair `pair`, copied into `labels` (DEVICE uint8
 * [H*W] of that pair's map) on the context stream, after that call's work.
 * Kept for pairs whose assignment ran in a fused multi-template launch
 * (refined search, BF16 or FP8 maps with D a multiple of 64 and aligned
 * rows, maps shared by at least two pairs); other pairs return
 * VQNNF_ENOTSUP (their label map is scratch reused pair by pair).  EINVAL
 * when `pair` is outside the last call.  Valid until the next batched call
 * on the context. */
vqnnf_status vqnnf_batched_labels(vqnnf_ctx* ctx, int32_t pair, uint8_t* labels);

/* Test support for the error bound of the refined search.  With a buffer
 * set, every refined matrix-core assignment on this context (BF16, FP32 and
 * FP8 maps; not the direct-distance path of D <= 32 or RGB maps) also writes
 * each pixel's FP32 scores s~_j = ||c_j||^2 - 2 q.c_j, the values the
 * error bound is applied to, to scores[pix * kpad + j] (DEVICE float,
 * kpad = k rounded up to a multiple of 16; entries j >= k are padding).  A
 * call whose map needs more than `capacity` floats returns EINVAL.  NULL
 * turns it off. */
vqnnf_status vqnnf_ctx_set_debug_scores(vqnnf_ctx* ctx, float* scores, int64_t capacity);

/* The error bound of the refined search for maps of storage `dtype`
 * (VQNNF_BF16, VQNNF_F32, or VQNNF_FP8_E4M3 with its HOST channel_scale[D]):
 * out[0..2] = a0, a1, a2 of the flag threshold
 * T(n) = a0 + n * (a1 + n * a2), n an upper bound of the pixel's norm (of
 * the stored values: the E4M3 codes' values for FP8 maps); out[3..4] = A0, A1
 * of the per-codeword score bound |s~_j - s_j| <= A0 + A1 * n that T is
 * built from (T also covers the FP64 rule's own rounding).  Host only. */
vqnnf_status vqnnf_template_score_bound(const vqnnf_template* t, int32_t dtype, const float* channel_scale,
                                        double* out);

/* Autotuning (1 = on, the default) of schedules that never change a result:
 *  - the refined assignment kernel's schedule, per shape class (D, padded
 *    codebook size, storage, map size to a power of two): the first refined
 *    call of a class times each schedule on its own data;
 *  - the on-chip score's tile block width (16 or 32 channels) and tile
 *    height, per shape (template size, grid, codebook size, map size; for a
 *    batched score launch, the shapes of all its pairs): the first call
 *    times both widths at a few heights on its own data.
 * Each candidate run writes the same labels / heatmap; the fastest is kept.
 * Calls made while a graph is captured (and vqnnf_match_noalloc) use tuned
 * values if there are any, else the defaults.  0 turns tuning off and
 * forgets tuned values. */
vqnnf_status vqnnf_ctx_set_autotune(vqnnf_ctx* ctx, int32_t enable);

/* Persists the context's tuning results in a text file (HOST path): entries
 * already in the file for this device's compute-unit count are loaded now,
 * and the file is rewritten (atomically, by rename) whenever tuning adds an
 * entry, so later processes skip the tuning runs.  NULL stops persisting;
 * results stay in memory.  A missing file is not an error; EINVAL when the
 * file cannot be written.  Lines are "<kind> <compute units> <shape key...>
 * <value>": kind a = assignment schedule, s = single-pair score tile, b =
 * batched score tile; a score tile value is the window rows per tile, plus
 * 65536 for 32-channel tile blocks. */
vqnnf_status vqnnf_ctx_set_tune_file(vqnnf_ctx* ctx, const char* path);

/* Graph mode for vqnnf_match_batched (0 = off, the default: kernels are
 * launched one by one).  Turning it off releases the captured graph. */
vqnnf_status vqnnf_ctx_set_graph(vqnnf_ctx* ctx, int32_t enable);

/* Per-kernel timing.  When enabled, the library brackets every kernel it
 * launches with HIP events on the context stream.  vqnnf_ctx_kernel_times
 * synchronises, then reports for each kernel name (up to max_entries)
 * the number of launches and their total duration in milliseconds since the
 * last reset.  names receives pointers to static strings. */
vqnnf_status vqnnf_ctx_set_timing(vqnnf_ctx* ctx, int32_t enable);
vqnnf_status vqnnf_ctx_kernel_times(vqnnf_ctx* ctx, int32_t max_entries, const char** names,
                                    int64_t* launches, double* total_ms, int32_t* n_entries);
vqnnf_status vqnnf_ctx_reset_times(vqnnf_ctx* ctx);

/* Description of the last error on the calling thread ("" if none). */
const char* vqnnf_last_error(void);

/* Library version string. */
const char* vqnnf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VQNNF_H */
