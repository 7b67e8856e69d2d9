// Internal declarations shared by the host API and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <deque>
#include <string>
#include <vector>

#include "../../include/vqnnf.h"

namespace vqnnf {

// Largest codebook the kernels handle (labels are uint8).
constexpr int kMaxK = 256;

// Assignment tiling: the codebook is padded to KPAD = 16 * KB codewords; the
// feature dimension is padded to a whole number of "load groups".  For the
// BF16 matrix-core path a load group is 32*S elements: lane group g of a
// 64-lane wave reads elements [8*S*g, 8*S*g + 8*S) of its pixel and feeds
// elements [8*S*g + 8*s, +8) to K-step s of the group; the codebook
// fragments are laid out on the host with the same element order.
struct AssignGeom {
  int kpad;        // codewords padded to a multiple of 16
  int kb;          // kpad / 16
  int s_bf16;      // K-steps (of 32 elements) per load group, 1, 2 or 4
  int d_pad_bf16;  // D padded to a multiple of 32 * s_bf16
  int e_f32;       // elements per lane per load group for the FP32 path (4 or 8)
  int d_pad_f32;   // D padded to a multiple of 4 * e_f32
};

AssignGeom make_assign_geom(int k, int D);

// Per-pixel error bound of the refined path: flag a pixel when
// s(2) - s(1) <= a0 + ||q|| * (a1 + ||q|| * a2), ||q|| an upper bound of the
// query pixel's norm; codeword j is a candidate when s_j - s(1) is within the
// same threshold.  Constants are rounded up.
struct BoundCoef {
  float a0, a1, a2;
  // host only: the per-codeword score bound behind the threshold,
  // |s~_j - s_j| <= A0 + A1 * ||q|| for every codeword j (before the FP64
  // rule's own rounding and the safety factors are added)
  double A0, A1;
};

// Filter geometry for the on-chip score kernel: the bank must be the full
// window plus one g x g grid over the full window (the benchmark bank).
struct GridBank {
  bool valid;
  int g;
  int xe[9];   // column edges X_0..X_g (X_0 = 0, X_g = w)
  int ye[9];   // row edges
};

// A bank with weighted filters, as the integral-image bank kernel reads it:
// region groups of up to kBankMaxG x kBankMaxG bins (the taps of Alg. 2's
// dilation filters sit on their edges) and filters that weigh a group's
// bins.  A weighted desc is one group with one filter; an indicator desc is
// one group whose every bin is a filter (coefficient 1), or, when its grid
// is larger than kBankMaxG, one 1 x 1 group per bin.
constexpr int kBankMaxG = 4;
// The bank kernel keeps the group table and every filter's R(tau), bin
// coefficients and weight (16 words per group + n_filters x (kpad + 17)
// floats) in LDS.
constexpr size_t kBankMaxLds = 160 * 1024;
struct BankGroup {      // 16 int32 on the device
  int32_t gx, gy;       // bins
  int32_t f0, f1;       // filters [f0, f1) weigh this group's bins
  int32_t xe[5], ye[5]; // tap offsets (bin edges) from the window's top-left;
                        // entries past gx / gy repeat the last edge
  int32_t pad[2];
};
static_assert(sizeof(BankGroup) == 64, "device layout");

// Assignment tables for FP8 maps of one channel-scale vector: the scale is
// folded into the codebook (c' = s*c), so they are built per distinct scale.
struct ScaledSet {
  std::vector<float> scale;          // the scales these tables belong to
  uint4* d_frag_bf16 = nullptr;      // fragments of c' (BF16 hi/lo), scaled by -2
  float* d_frag_f32 = nullptr;       // fragments of c' (FP32), scaled by -2
  float* d_scale = nullptr;          // [D] device copy of the scales
  BoundCoef bound{};
};

struct DeviceTemplate {
  int w = 0, h = 0, D = 0, k = 0, n_filters = 0;
  AssignGeom geom{};
  // host copies
  std::vector<float> codebook;       // [k][D]
  std::vector<uint8_t> labels;       // [h][w]
  std::vector<int32_t> counts;       // [n_filters][k]
  std::vector<float> weights;        // [n_filters]
  // expanded filter boxes (template coordinates), one per filter
  std::vector<int32_t> boxes;        // [n_filters][4] x0,y0,x1,y1 (indicator banks)
  GridBank grid{};
  // banks with weighted filters (scored by the bank kernel)
  bool weighted = false;
  int bank_g = 0;                    // largest group side (1..kBankMaxG)
  std::vector<BankGroup> groups;
  std::vector<float> coef;           // [n_filters][16]: bin (a, b) at b * 4 + a
  std::vector<float> resp;           // [n_filters][k] R(tau), FP32 as the kernel computes it
  BoundCoef bound_bf16q{};           // BF16-stored query, codebook hi+lo
  BoundCoef bound_f32q{};            // FP32-stored query, both split hi+lo
  std::vector<float> cnorm32;        // [k] ||c||^2 rounded to FP32
  // FP8 tables, one per distinct scale vector; a deque keeps every set at a
  // fixed address while more are added (callers hold pointers to them)
  std::deque<ScaledSet> scaled;
  // device copies
  void* d_blob = nullptr;            // one allocation holding every table below
  float* d_codebook = nullptr;       // [k][D] FP32
  uint4* d_frag_bf16 = nullptr;      // A fragments, BF16 hi/lo, scaled by -2
  float* d_frag_f32 = nullptr;       // A fragments, FP32, scaled by -2
  float* d_cnorm = nullptr;          // [kpad] ||c||^2 (pad: 3e38)
  int32_t* d_counts = nullptr;       // [n_filters][kpad] (pad channels 0)
  uint32_t* d_counts16 = nullptr;    // [n_filters][kpad/2] u16 pairs
  float* d_weights = nullptr;        // [n_filters]
  int32_t* d_boxes = nullptr;        // [n_filters][4]
  BankGroup* d_groups = nullptr;     // weighted banks
  float* d_coef = nullptr;           // [n_filters][16]
  float* d_resp = nullptr;           // [n_filters][kpad] (pad channels 0)
  int magic = 0;
};

// ---------------------------------------------------------------- host prep
std::vector<double> kmeans_host(const std::vector<double>& x, int64_t n, int D, int k, int iters,
                                uint64_t seed);
std::vector<int> assign_host(const std::vector<double>& x, int64_t n, int D,
                             const std::vector<double>& c, int k);
// Template NNF and R(tau) on the host; `labels` (h*w, optional) is the NNF
// already computed on the device.
void rgb_patch_features_host(const uint8_t* img, int H, int W, int64_t stride, float* out);
// PCA of n points (row stride `stride` floats): mean, the d principal axes
// (rows, largest-magnitude component positive) and their variances, FP64.
void pca_fit_host(const float* x, int64_t n, int64_t stride, int D, int d, std::vector<double>& mean,
                  std::vector<double>& basis, std::vector<double>& var);
void prepare_template_host(DeviceTemplate& t, const float* tmpl, int64_t tmpl_stride,
                           const uint8_t* labels = nullptr);

// Device-ready tables of a template, built on the host.
struct HostTables {
  std::vector<uint16_t> frag_bf16;   // [steps][2][kb][64][8]
  std::vector<float> frag_f32;       // [steps][kb][64]
  std::vector<float> cnorm;          // [kpad]
  std::vector<int32_t> counts;       // [nf][kpad]
  std::vector<uint32_t> counts16;    // [nf][kpad/2]
  std::vector<float> resp;           // [nf][kpad] weighted banks
};
void build_tables(DeviceTemplate& t, HostTables& ht);
void build_scaled_tables(const DeviceTemplate& t, const float* scale, std::vector<uint16_t>& frag_bf16,
                         std::vector<float>& frag_f32, BoundCoef& bound);

// ---------------------------------------------------------------- launches
// All launchers enqueue on `stream` and return hipSuccess or the first error.

struct AssignArgs {
  const void* q;
  int64_t stride;        // elements between pixels
  int64_t n_pix;         // H * W
  int D;
  int dtype;             // vqnnf_dtype
  const DeviceTemplate* t;
  const uint4* frag_bf16;  // codebook fragments (the template's, or its FP8 ScaledSet's)
  const float* frag_f32;
  const float* scale;      // FP8 maps: [D] device channel scales; else null
  int img_w, img_h;        // RGB maps: image size (colour features built per pixel)
  uint8_t* labels;
  // refined path only
  uint32_t* wl_count;    // worklist counter (must be 0 on entry)
  uint32_t* wl_pix;      // [n_pix]
  uint32_t* wl_mask;     // [n_pix][mask_words]
  int mask_words;        // 0: ceil(kpad / 32); the fused multi-template kernel writes its own count
  BoundCoef bound;
  float* dump;           // refined matrix-core path, test support: s~ [n_pix][kpad] or null
  int variant;           // refined matrix-core path: schedule 1..refined_variants(), 0 = default
};

// Fused assignment of several templates against one map (batched matching).
constexpr int kMultiMaxPass = 96;    // passes of 128 codewords per launch (norms in LDS)
struct MultiPass {                   // one pass: n_seg templates of sb blocks each
  int sb, tmpl0, n_seg, pad;
};
struct MultiOut {                    // per template: outputs and error bound
  uint8_t* labels;
  uint32_t* wl_count;
  uint32_t* wl_pix;
  uint32_t* wl_mask;                 // [n_pix][(sb+1)/2]
  float a0, a1, a2, pad;
};
// One query map of a fused launch: its templates' pass plan and outputs.
struct MultiMap {
  const void* q;
  int64_t stride;
  int64_t n_pix;
  const uint4* frag;                 // [n_pass][n_groups][2][8][64] BF16 fragment pairs
  const float* cnorm;                // [n_pass][128] ||c||^2 (pad 3e38)
  const MultiPass* passes;
  const MultiOut* outs;
  int n_pass, pad;
  int64_t tile0;                     // first tile of the map in the launch's tile list
};
struct MultiParams {
  const MultiMap* maps;              // device table, tile0 ascending
  int n_maps;
  int D, n_groups;                   // shared by every map of the launch
  int64_t n_tiles;                   // all maps
};
struct MultiArgs {
  MultiParams kp;
  bool fp8;
  int variant;                       // 0/1 the compiler's schedule, 2 fragments one block ahead
};
// Pixels per tile of the fused launch and the tiles of one map.
constexpr int kMultiTilePx = 512;
__host__ __device__ inline int64_t multi_tiles(int64_t n_pix) {
  return (n_pix + kMultiTilePx - 1) / kMultiTilePx;
}
hipError_t launch_assign_multi(const MultiArgs& a, hipStream_t s, int n_cu);

hipError_t launch_assign_plain(const AssignArgs& a, hipStream_t s, int n_cu);
hipError_t launch_assign_refined(const AssignArgs& a, hipStream_t s, int n_cu);
// Schedules of the refined kernel available for these arguments (1 or 2);
// the highest is the default.
int refined_variants(const AssignArgs& a);
hipError_t launch_rescore(const AssignArgs& a, hipStream_t s, int n_cu);
// Batched re-score of many pairs: one launch per (query type, vector path)
// class, each pair's arguments read from a device table.
struct RescoreBatchPlan {
  struct Launch {
    int qt, vec;
    size_t tab_off;
    int n;
  };
  std::vector<uint8_t> blob;
  std::vector<Launch> launches;
};
void plan_rescore_batch(const std::vector<AssignArgs>& pairs, RescoreBatchPlan* out);
hipError_t launch_rescore_batch(const RescoreBatchPlan& plan, const uint8_t* d_blob, int n_cu, hipStream_t s);
// Low-dimensional features (F32 / BF16, D <= 32) and RGB colour features:
// direct FP32 distances with a relative error bound; `refined` appends
// near ties to the re-score worklist.
bool lowd_supported(int dtype, int D);
// Projection onto d <= 64 principal axes (device tables: basis t-major
// [D][d], mean [D], FP8 channel scales [D]).
hipError_t launch_pca_project(const void* q, int dtype, int64_t stride, int H, int W, int D, const float* scale,
                              const float* mean, const float* basis_t, int d, float* out, hipStream_t s);
// BF16 maps, D a multiple of 32, 16-byte aligned rows: matrix cores with the
// basis split into three exact BF16 terms (fragments [D/32][3][ceil(d/16)][64]
// uint4) and the centring mean . basis subtracted at the end.
size_t pca_mfma_lds(int D, int d);
hipError_t launch_pca_mfma(const uint16_t* q, int64_t stride, int H, int W, int D, const uint4* frag,
                           const float* mb, int d, float* out, int n_cu, hipStream_t s);
hipError_t launch_assign_lowd(const AssignArgs& a, bool refined, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);

struct IntegralArgs {
  const uint8_t* labels;
  int H, W, k;
  int32_t* P;            // [(H+1)(W+1)k]
  uint16_t* P16;         // if set, P is written here instead, mod 2^16
  int32_t* rsh;          // [H][S][k]
  int32_t* cbh;          // [R][W][k]
  int32_t* th;           // [R][S][k]
};
constexpr int kIntTile = 64;
hipError_t launch_integral(const IntegralArgs& a, hipStream_t s);

struct ScoreArgs {
  const DeviceTemplate* t;
  const uint8_t* labels;       // on-chip path
  const int32_t* P;            // integral path
  const uint16_t* P16;         // weighted banks: integral image mod 2^16, even channel count
  int H, W;
  float* heatmap;
  unsigned long long* best;    // packed (orderable score, ~index), must be 0
  void* partials;              // on-chip path: per channel group partial sums
  int n_cu;                    // compute units (tile sizing)
  int tyw;                     // on-chip path: window rows per tile, 0 = default sizing
  int kgsel;                   // on-chip path: channels per tile block, 0 = default rule,
                               // 1 = 16, 2 = 32 where the grid allows
};
hipError_t launch_score_fused(const ScoreArgs& a, hipStream_t s, size_t* lds_bytes_out);
hipError_t launch_score_integral(const ScoreArgs& a, hipStream_t s);
// Weighted banks: heatmap + best from the integral image a.P.
hipError_t launch_score_bank(const ScoreArgs& a, hipStream_t s);
// Batched on-chip score of many (template, label map) pairs: one tile launch
// per (grid size, uniform bins) class and one combine launch per stored-sum
// layout, each reading its pairs' arguments from a device table.
struct ScoreBatchItem {
  const DeviceTemplate* t;
  const uint8_t* labels;
  int H, W;
  float* heatmap;
  unsigned long long* best;    // must be 0
  int tyw;                     // window rows per tile (>= 1)
};
struct ScoreBatchLaunch {
  int kind;                    // 0 tile, 1 combine
  int G, uni, kg, nacc;        // kg: channels per tile block
  int sad;                     // tile blocks sum |T_j - C_j|
  size_t tab_off, blk_off;     // byte offsets into the table blob
  uint32_t nblk;
};
struct ScoreBatchPlan {
  std::vector<uint8_t> blob;   // argument tables and block -> pair maps
  std::vector<ScoreBatchLaunch> launches;
  size_t part_bytes = 0;       // partial sums of all pairs
};
// Plans the launches with the partial sums placed in `part` (nullptr: sizes
// only).  False when a pair's bank is not on-chip or a size overflows.
// wide: 32-channel tile blocks for the pairs whose grid allows them.
bool plan_score_batch(const std::vector<ScoreBatchItem>& items, void* part, ScoreBatchPlan* out,
                      bool wide = false);
// d_blob: a device copy of plan.blob.
hipError_t launch_score_batch(const ScoreBatchPlan& plan, const uint8_t* d_blob, hipStream_t s);
// True when the on-chip score kernel can take this template's bank.
bool fused_supported(const DeviceTemplate& t);
// The on-chip score can use 32-channel tile blocks for this template; and
// whether a single pair uses them by default.
bool fused_wide_allowed(const DeviceTemplate& t);
bool fused_default_wide(const DeviceTemplate& t);
int fused_groups(const DeviceTemplate& t);   // channel groups of the tile score
// Scratch bytes of the on-chip path's per-channel-group partial sums.
size_t fused_partial_bytes(const DeviceTemplate& t, int H, int W);
// Default window rows per tile of the on-chip score for this shape and
// block width.
int fused_default_tyw(const DeviceTemplate& t, int H, int W, int n_cu, bool wide);
hipError_t launch_zero_u64(unsigned long long* p, hipStream_t s);

// k-means of one template's points on the device (all buffers device).
struct KmJob {
  const float* x;        // [l][D] points, FP32
  float* xt;             // [D][l] the same, dimension-major
  double* c;             // [k][D] centres
  float* c32;            // [k][D] final codebook
  uint8_t* lab;          // [l] labels (after the call: NNF against c32)
  int* idx;              // [l] points grouped by cluster, in point order
  int* start;            // [k + 1] cluster offsets into idx
  double* d2;            // [l] k-means++ D^2
  uint64_t* state;       // [1] generator state between draws
  double* pdist;         // [ceil(k/16)][l] nearest distance per centre chunk
  uint8_t* pidx;         // [ceil(k/16)][l] its centre
  uint64_t seed;
  int l, D, k, pad;
};
hipError_t launch_kmeans(const KmJob* d_jobs, const std::vector<KmJob>& jobs, int iters, hipStream_t s);

// Fixed scratch of vqnnf_match_noalloc: a static device array of this size
// per device.  noalloc_scratch_init (device current) resolves its address
// once per device; noalloc_scratch returns it (null before the init).
constexpr size_t kNoAllocScratchBytes = (size_t)VQNNF_NOALLOC_SCRATCH_BYTES;
hipError_t noalloc_scratch_init(int device);
void* noalloc_scratch(int device);

// Kernel-name registry for timing.
enum KernelId {
  K_FILL = 0, K_ASSIGN_PLAIN, K_ASSIGN_REFINED, K_RESCORE, K_INT_EDGE, K_INT_PREFIX,
  K_INT_MAIN, K_SCORE_FUSED, K_SCORE_COMBINE, K_SCORE_INTEGRAL, K_ASSIGN_MULTI, K_SCORE_BANK,
  K_KMEANS, K_ASSIGN_LOWD, K_PCA_PROJECT, K_COUNT
};
const char* kernel_name(int id);

// Timing hook: the launchers call these around each kernel when timing is on.
struct TimingHook {
  void (*begin)(void* user, int kernel_id);
  void (*end)(void* user, int kernel_id);
  void* user;
};
void set_timing_hook(const TimingHook* h);   // thread-local
void timing_begin(int id);
void timing_end(int id);

}  // namespace vqnnf
