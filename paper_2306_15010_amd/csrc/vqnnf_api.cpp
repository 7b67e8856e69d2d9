// C ABI of the VQ-NNF library: contexts, templates, validation, scratch
// management, timing and the orchestration of the gfx950 kernels.
#pragma clang fp contract(off)

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <map>
#include <thread>
#include <vector>

#include "vqnnf_internal.h"

using namespace vqnnf;

namespace {

thread_local std::string g_err;

vqnnf_status fail(vqnnf_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

vqnnf_status ok() { return VQNNF_OK; }

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(VQNNF_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));                \
  } while (0)

constexpr int kCtxMagic = 0x51CE7001;
constexpr int kTplMagic = 0x7E3B1A7E;
// tuned score tile choice: window rows per tile, this bit set for 32-channel
// tile blocks
constexpr int kScoreWide = 1 << 16;

struct Buffer {
  void* p = nullptr;
  size_t bytes = 0;
};

struct TimingRecord {
  int id;
  hipEvent_t a, b;
};

}  // namespace

struct vqnnf_ctx {
  int magic = kCtxMagic;
  bool has_device = false;
  int device = -1;
  int n_cu = 256;
  hipStream_t stream = nullptr;
  uint64_t cap = 0;
  uint64_t used = 0;
  // scratch
  Buffer control;      // [0]: u64 best, [8]: u32 worklist count
  Buffer labels;       // uint8 [n_pix]
  Buffer wl_pix;       // u32 [n_pix]
  Buffer wl_mask;      // u32 [n_pix][mask_words]
  Buffer int_side;     // integral side arrays
  Buffer int_p;        // integral image for the integral score path
  Buffer partials;     // per channel group partial sums of the on-chip score
  Buffer keys;         // u64 [n_pairs] best keys of a batched call
  Buffer pca;          // projection tables: basis, mean, channel scales
  // fused multi-template assignment of a batch (per map group)
  Buffer m_labels;     // uint8 [n_templates][n_pix]
  Buffer m_count;      // u32 [n_templates] worklist counters
  Buffer m_wl_pix;     // u32 [n_templates][n_pix]
  Buffer m_wl_mask;    // u32 [n_templates][n_pix][4]
  struct MultiPlan {
    std::vector<uint64_t> sig;
    Buffer frag, cnorm, passes, outs;
    int n_pass = 0;
    int n_groups = 0;                  // load groups of 32 elements along D
    std::vector<int> slot_pair;        // output slot -> index in the map group
  };
  std::vector<MultiPlan> mplans;       // one per map group of the last batch
  // label map (and its size) of every pair of the last batch whose
  // assignment ran fused; null for the others
  std::vector<std::pair<const uint8_t*, int64_t>> batch_labels;
  // batched re-score and score of the fused groups' pairs
  Buffer b_part;       // partial sums of every pair's on-chip score
  Buffer b_tab;        // argument tables (re-score, then score)
  std::vector<uint8_t> b_tab_host;     // what b_tab holds
  void* b_tab_at = nullptr;            // ... at this allocation
  std::map<std::vector<int>, int> btyw_cache;   // batch shapes -> score tile choice
  // autotuned score tile choice (window rows per tile, kScoreWide), by shape
  // (w, h, g, kpad, H, W, uniform bins)
  bool autotune = true;
  bool capturing = false;
  std::map<std::vector<int>, int> tyw_cache;
  // batched calls captured into a graph (vqnnf_ctx_set_graph)
  bool graph = false;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<uint64_t> gsig;
  // refined assignment schedule: 0 = tuned per shape class (default when
  // tuning is off); VQNNF_ASSIGN_VARIANT forces one when the context is made
  int assign_variant = 0;
  std::map<std::vector<int>, int> avar_cache;   // shape class -> schedule
  std::string tune_file;                        // persisted tuning results, "" = none
  // test support: scores of the refined matrix-core assignment
  float* dbg_scores = nullptr;
  int64_t dbg_cap = 0;
  // timing
  bool timing = false;
  std::vector<TimingRecord> pending;
  std::vector<hipEvent_t> pool;
  int64_t launches[K_COUNT] = {};
  double total_ms[K_COUNT] = {};
};

// Every template gets an id that is never reused, so plans and graphs keyed
// on it cannot match a later template that happens to get the same address.
std::atomic<uint64_t> g_next_template_uid{1};

struct vqnnf_template {
  int magic = kTplMagic;
  vqnnf_ctx* ctx = nullptr;
  uint64_t uid = g_next_template_uid.fetch_add(1);
  DeviceTemplate t;
};

namespace {

// ---------------------------------------------------------------- timing
void hook_begin(void* user, int id) {
  auto* c = (vqnnf_ctx*)user;
  TimingRecord r{id, nullptr, nullptr};
  if (c->pool.size() >= 2) {
    r.a = c->pool.back(); c->pool.pop_back();
    r.b = c->pool.back(); c->pool.pop_back();
  } else {
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return;
  }
  hipEventRecord(r.a, c->stream);
  c->pending.push_back(r);
}
void hook_end(void* user, int id) {
  auto* c = (vqnnf_ctx*)user;
  if (c->pending.empty() || c->pending.back().id != id) return;
  hipEventRecord(c->pending.back().b, c->stream);
}

struct HookScope {
  bool on;
  explicit HookScope(vqnnf_ctx* c) : on(c->timing) {
    if (on) {
      TimingHook h{hook_begin, hook_end, c};
      set_timing_hook(&h);
    }
  }
  ~HookScope() {
    if (on) set_timing_hook(nullptr);
  }
};

vqnnf_status collect_times(vqnnf_ctx* c) {
  if (c->pending.empty()) return ok();
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (auto& r : c->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      c->launches[r.id] += 1;
      c->total_ms[r.id] += ms;
    }
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->pending.clear();
  return ok();
}

// ---------------------------------------------------------------- scratch
vqnnf_status ensure(vqnnf_ctx* c, Buffer& b, size_t bytes, const char* what) {
  if (bytes <= b.bytes) return ok();
  size_t grow = std::max(bytes, b.bytes + b.bytes / 4);
  grow = (grow + 255) & ~size_t(255);
  uint64_t after = c->used - b.bytes + grow;
  if (after > c->cap) {
    grow = (bytes + 255) & ~size_t(255);
    after = c->used - b.bytes + grow;
    if (after > c->cap)
      return fail(VQNNF_ENOMEM, "%s needs %zu bytes of scratch; the context cap is %llu bytes "
                  "(%llu in use)", what, bytes, (unsigned long long)c->cap,
                  (unsigned long long)(c->used - b.bytes));
  }
  if (!c->has_device)
    return fail(VQNNF_ENOTSUP, "context has no device (created with vqnnf_ctx_create_host)");
  if (b.p) {
    // the stream may still use the old buffer
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipFree(b.p));
    c->used -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
  }
  hipError_t e = hipMalloc(&b.p, grow);
  if (e != hipSuccess) {
    b.p = nullptr;
    return fail(VQNNF_ENOMEM, "hipMalloc(%zu) for %s failed: %s", grow, what, hipGetErrorString(e));
  }
  b.bytes = grow;
  c->used += grow;
  return ok();
}

// Checks scratch needs against the cap before anything is enqueued.
vqnnf_status check_cap(vqnnf_ctx* c, std::initializer_list<std::pair<const Buffer*, size_t>> need) {
  uint64_t total = c->used;
  for (auto& n : need)
    if (n.second > n.first->bytes) total = total - n.first->bytes + ((n.second + 255) & ~size_t(255));
  if (total > c->cap)
    return fail(VQNNF_ENOMEM, "call needs %llu bytes of scratch in total; the context cap is %llu",
                (unsigned long long)total, (unsigned long long)c->cap);
  return ok();
}

// ---------------------------------------------------------------- validation
vqnnf_status check_ctx(const vqnnf_ctx* c) {
  if (!c) return fail(VQNNF_EHANDLE, "null context");
  if (c->magic != kCtxMagic) return fail(VQNNF_EHANDLE, "invalid or destroyed context");
  return ok();
}

vqnnf_status check_tpl(const vqnnf_ctx* c, const vqnnf_template* t) {
  if (!t) return fail(VQNNF_EHANDLE, "null template");
  if (t->magic != kTplMagic) return fail(VQNNF_EHANDLE, "invalid or freed template");
  if (c && t->ctx != c) return fail(VQNNF_EINVAL, "template belongs to another context");
  return ok();
}

size_t dtype_size(int dt) {
  switch (dt) {
    case VQNNF_F32: return 4;
    case VQNNF_BF16: return 2;
    case VQNNF_FP8_E4M3: return 1;
    case VQNNF_RGB8: return 1;
  }
  return 0;
}

// BF16 rounding (nearest, ties to even) of a finite FP32 value, and its bits.
uint16_t bf16_bits(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float bf16_round(float x) {
  const uint32_t u = (uint32_t)bf16_bits(x) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// Elements between pixels (bytes for an RGB image, whose pixel is 3 bytes).
int64_t map_stride(const vqnnf_fmap* m) {
  if (m->pixel_stride) return m->pixel_stride;
  return m->dtype == VQNNF_RGB8 ? 3 : m->D;
}

vqnnf_status check_map(const vqnnf_fmap* m, const char* what) {
  if (!m) return fail(VQNNF_EINVAL, "%s: null map", what);
  if (!m->data) return fail(VQNNF_EINVAL, "%s: null data pointer", what);
  if (dtype_size(m->dtype) == 0) return fail(VQNNF_EINVAL, "%s: unknown dtype %d", what, m->dtype);
  if (m->H < 1 || m->W < 1) return fail(VQNNF_EINVAL, "%s: H and W must be >= 1 (got %d x %d)", what, m->H, m->W);
  if (m->D < 1) return fail(VQNNF_EINVAL, "%s: D must be >= 1 (got %d)", what, m->D);
  const int64_t st = map_stride(m);
  if (m->dtype == VQNNF_RGB8) {
    if (m->D != 27) return fail(VQNNF_EINVAL, "%s: an RGB map has D = 27 colour features (got %d)", what, m->D);
    if (st < 3) return fail(VQNNF_EINVAL, "%s: RGB pixel_stride %lld < 3 bytes", what, (long long)st);
  } else if (st < m->D) {
    return fail(VQNNF_EINVAL, "%s: pixel_stride %lld < D %d", what, (long long)st, m->D);
  }
  if ((int64_t)m->H * m->W >= (1ll << 31)) return fail(VQNNF_EINVAL, "%s: H*W must be < 2^31", what);
  if (st * (int64_t)dtype_size(m->dtype) > (1ll << 22))
    return fail(VQNNF_EINVAL, "%s: a pixel row (pixel_stride * element size) must be <= 4 MiB", what);
  if (m->dtype == VQNNF_FP8_E4M3) {
    if (!m->channel_scale) return fail(VQNNF_EINVAL, "%s: FP8 map needs channel_scale", what);
    for (int d = 0; d < m->D; ++d)
      if (!std::isfinite(m->channel_scale[d]) || m->channel_scale[d] < 0.0f)
        return fail(VQNNF_EINVAL, "%s: channel_scale[%d] must be finite and >= 0", what, d);
  }
  return ok();
}

// Banks with weighted filters: region groups for the bank kernel (see
// BankGroup); filters in desc order, a desc's bins row-major, as for
// indicator banks.  Consecutive weighted descs over the same region and grid
// (the filters of one scale) share one group.
void expand_weighted(const vqnnf_filter_desc* bank, int n_desc, DeviceTemplate& t) {
  t.groups.clear();
  t.coef.clear();
  t.weights.clear();
  auto edge = [](int lo, int hi, int g, int a) { return lo + (int)((int64_t)a * (hi - lo) / g); };
  auto add_filter = [&](double weight) {
    t.coef.resize(t.coef.size() + 16, 0.0f);
    t.weights.push_back((float)weight);
    return (int)t.weights.size() - 1;
  };
  for (int i = 0; i < n_desc; ++i) {
    const vqnnf_filter_desc& d = bank[i];
    const bool small = d.gx <= kBankMaxG && d.gy <= kBankMaxG;
    if (d.bin_weight && i > 0 && bank[i - 1].bin_weight && bank[i - 1].x0 == d.x0 &&
        bank[i - 1].y0 == d.y0 && bank[i - 1].x1 == d.x1 && bank[i - 1].y1 == d.y1 &&
        bank[i - 1].gx == d.gx && bank[i - 1].gy == d.gy) {
      // same region and grid as the previous weighted desc: its group's
      // bin counts serve this filter too
      BankGroup& g = t.groups.back();
      const double region = (double)(d.x1 - d.x0) * (double)(d.y1 - d.y0);
      const int f = add_filter((double)d.weight);
      for (int b = 0; b < d.gy; ++b)
        for (int a = 0; a < d.gx; ++a)
          t.coef[(size_t)f * 16 + b * 4 + a] = (float)((double)d.bin_weight[b * d.gx + a] / region);
      g.f1 = f + 1;
      continue;
    }
    if (d.bin_weight || small) {
      BankGroup g{};
      g.gx = d.gx;
      g.gy = d.gy;
      for (int a = 0; a <= d.gx; ++a) g.xe[a] = edge(d.x0, d.x1, d.gx, a);
      for (int b = 0; b <= d.gy; ++b) g.ye[b] = edge(d.y0, d.y1, d.gy, b);
      g.f0 = (int)t.weights.size();
      if (d.bin_weight) {
        const double region = (double)(d.x1 - d.x0) * (double)(d.y1 - d.y0);
        const int f = add_filter((double)d.weight);
        for (int b = 0; b < d.gy; ++b)
          for (int a = 0; a < d.gx; ++a)
            t.coef[(size_t)f * 16 + b * 4 + a] = (float)((double)d.bin_weight[b * d.gx + a] / region);
      } else {
        for (int b = 0; b < d.gy; ++b)
          for (int a = 0; a < d.gx; ++a) {
            const double area = (double)(g.xe[a + 1] - g.xe[a]) * (double)(g.ye[b + 1] - g.ye[b]);
            const int f = add_filter((double)d.weight / ((double)d.gx * d.gy * area));
            t.coef[(size_t)f * 16 + b * 4 + a] = 1.0f;
          }
      }
      g.f1 = (int)t.weights.size();
      t.groups.push_back(g);
    } else {
      for (int b = 0; b < d.gy; ++b)
        for (int a = 0; a < d.gx; ++a) {
          BankGroup g{};
          g.gx = g.gy = 1;
          g.xe[0] = edge(d.x0, d.x1, d.gx, a);
          g.xe[1] = edge(d.x0, d.x1, d.gx, a + 1);
          g.ye[0] = edge(d.y0, d.y1, d.gy, b);
          g.ye[1] = edge(d.y0, d.y1, d.gy, b + 1);
          const double area = (double)(g.xe[1] - g.xe[0]) * (double)(g.ye[1] - g.ye[0]);
          g.f0 = add_filter((double)d.weight / ((double)d.gx * d.gy * area));
          g.f1 = g.f0 + 1;
          t.coef[(size_t)g.f0 * 16] = 1.0f;
          t.groups.push_back(g);
        }
    }
  }
  t.n_filters = (int)t.weights.size();
  // edges past a group's grid repeat its last edge (zero-area bins the
  // kernel's fixed tap pattern can read); largest side for the kernel shape
  t.bank_g = 1;
  for (BankGroup& g : t.groups) {
    for (int a = g.gx + 1; a <= kBankMaxG; ++a) g.xe[a] = g.xe[g.gx];
    for (int b = g.gy + 1; b <= kBankMaxG; ++b) g.ye[b] = g.ye[g.gy];
    t.bank_g = std::max(t.bank_g, std::max(g.gx, g.gy));
  }
}

vqnnf_status expand_bank(const vqnnf_filter_desc* bank, int n_desc, int w, int h,
                         DeviceTemplate& t) {
  if (!bank || n_desc < 1) return fail(VQNNF_EINVAL, "filter bank: need n_desc >= 1 and a bank pointer");
  bool weighted = false;
  for (int i = 0; i < n_desc; ++i) {
    const vqnnf_filter_desc& d = bank[i];
    if (d.x0 < 0 || d.y0 < 0 || d.x1 > w || d.y1 > h || d.x0 >= d.x1 || d.y0 >= d.y1)
      return fail(VQNNF_EINVAL, "filter %d: region [%d,%d)x[%d,%d) not inside the %dx%d template",
                  i, d.x0, d.x1, d.y0, d.y1, w, h);
    if (d.gx < 1 || d.gy < 1 || d.gx > d.x1 - d.x0 || d.gy > d.y1 - d.y0)
      return fail(VQNNF_EINVAL, "filter %d: grid %dx%d leaves empty bins", i, d.gx, d.gy);
    if (!std::isfinite(d.weight)) return fail(VQNNF_EINVAL, "filter %d: weight not finite", i);
    if (d.bin_weight) {
      if (d.gx > kBankMaxG || d.gy > kBankMaxG)
        return fail(VQNNF_ENOTSUP, "filter %d: weighted grids are at most %dx%d (got %dx%d)", i,
                    kBankMaxG, kBankMaxG, d.gx, d.gy);
      for (int b = 0; b < d.gx * d.gy; ++b)
        if (!std::isfinite(d.bin_weight[b]))
          return fail(VQNNF_EINVAL, "filter %d: bin_weight[%d] not finite", i, b);
      weighted = true;
    }
  }
  t.boxes.clear();
  t.weights.clear();
  t.groups.clear();
  t.coef.clear();
  t.weighted = weighted;
  if (weighted) {
    expand_weighted(bank, n_desc, t);
    const size_t lds = (t.groups.size() * 16 + (size_t)t.n_filters * (make_assign_geom(t.k, 1).kpad + 17)) *
                       sizeof(float);
    if (lds > kBankMaxLds)
      return fail(VQNNF_ENOTSUP, "weighted bank: %d filters x %d channels exceed the %zu KiB the bank "
                  "kernel holds on chip", t.n_filters, t.k, kBankMaxLds / 1024);
    t.grid = GridBank{};
    t.grid.valid = false;
    return ok();
  }
  for (int i = 0; i < n_desc; ++i) {
    const vqnnf_filter_desc& d = bank[i];
    for (int b = 0; b < d.gy; ++b)
      for (int a = 0; a < d.gx; ++a) {
        int bx0 = d.x0 + (int)((int64_t)a * (d.x1 - d.x0) / d.gx);
        int bx1 = d.x0 + (int)((int64_t)(a + 1) * (d.x1 - d.x0) / d.gx);
        int by0 = d.y0 + (int)((int64_t)b * (d.y1 - d.y0) / d.gy);
        int by1 = d.y0 + (int)((int64_t)(b + 1) * (d.y1 - d.y0) / d.gy);
        double area = (double)(bx1 - bx0) * (double)(by1 - by0);
        double wt = (double)d.weight / ((double)d.gx * d.gy * area);
        t.boxes.insert(t.boxes.end(), {bx0, by0, bx1, by1});
        t.weights.push_back((float)wt);
      }
  }
  t.n_filters = (int)t.weights.size();
  // Is it the full window plus one g x g grid over the full window?
  GridBank gb{};
  gb.valid = false;
  if (n_desc == 2 && bank[0].x0 == 0 && bank[0].y0 == 0 && bank[0].x1 == w && bank[0].y1 == h &&
      bank[0].gx == 1 && bank[0].gy == 1 && bank[1].x0 == 0 && bank[1].y0 == 0 &&
      bank[1].x1 == w && bank[1].y1 == h && bank[1].gx == bank[1].gy && bank[1].gx >= 1 &&
      bank[1].gx <= 4) {
    gb.valid = true;
    gb.g = bank[1].gx;
    for (int a = 0; a <= gb.g; ++a) {
      gb.xe[a] = (int)((int64_t)a * w / gb.g);
      gb.ye[a] = (int)((int64_t)a * h / gb.g);
    }
  }
  t.grid = gb;
  return ok();
}

template <typename T>
vqnnf_status upload(vqnnf_ctx* c, T** dst, const std::vector<T>& src) {
  *dst = nullptr;
  if (src.empty()) return ok();
  HIP_TRY(hipMalloc((void**)dst, sizeof(T) * src.size()));
  HIP_TRY(hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
  return ok();
}

void free_device(DeviceTemplate& t) {
  if (t.d_blob) hipFree(t.d_blob);
  t.d_blob = nullptr;
  t.d_codebook = nullptr; t.d_frag_bf16 = nullptr; t.d_frag_f32 = nullptr; t.d_cnorm = nullptr;
  t.d_counts = nullptr; t.d_counts16 = nullptr; t.d_weights = nullptr; t.d_boxes = nullptr;
  t.d_groups = nullptr; t.d_coef = nullptr; t.d_resp = nullptr;
  for (ScaledSet& ss : t.scaled) {
    if (ss.d_frag_bf16) hipFree(ss.d_frag_bf16);
    if (ss.d_frag_f32) hipFree(ss.d_frag_f32);
    if (ss.d_scale) hipFree(ss.d_scale);
  }
  t.scaled.clear();
}

// The FP8 tables of template t for the map's channel scales: found by value,
// else built on the host and uploaded (synchronously, before any launch that
// reads them).  Sets are kept for the life of the template.
vqnnf_status prepare_scaled(vqnnf_ctx* c, const vqnnf_template* tp, const vqnnf_fmap* q,
                            const ScaledSet** out) {
  *out = nullptr;
  if (q->dtype != VQNNF_FP8_E4M3) return ok();
  DeviceTemplate& t = const_cast<vqnnf_template*>(tp)->t;
  const int D = t.D;
  for (const ScaledSet& ss : t.scaled)
    if (std::memcmp(ss.scale.data(), q->channel_scale, sizeof(float) * D) == 0) {
      *out = &ss;
      return ok();
    }
  ScaledSet ss;
  ss.scale.assign(q->channel_scale, q->channel_scale + D);
  std::vector<uint16_t> fb16;
  std::vector<float> ff;
  build_scaled_tables(t, q->channel_scale, fb16, ff, ss.bound);
  std::vector<uint4> fb(fb16.size() / 8);
  std::memcpy(fb.data(), fb16.data(), fb16.size() * 2);
  vqnnf_status s;
  if ((s = upload(c, &ss.d_frag_bf16, fb)) || (s = upload(c, &ss.d_frag_f32, ff)) ||
      (s = upload(c, &ss.d_scale, ss.scale))) {
    if (ss.d_frag_bf16) hipFree(ss.d_frag_bf16);
    if (ss.d_frag_f32) hipFree(ss.d_frag_f32);
    if (ss.d_scale) hipFree(ss.d_scale);
    return s;
  }
  t.scaled.push_back(std::move(ss));
  *out = &t.scaled.back();
  return ok();
}

vqnnf_status finish_template(vqnnf_ctx* ctx, vqnnf_template* tp, const vqnnf_fmap* tmpl,
                             const uint8_t* labels = nullptr) {
  DeviceTemplate& t = tp->t;
  const float* td = (const float*)tmpl->data;
  int64_t st = tmpl->pixel_stride ? tmpl->pixel_stride : tmpl->D;
  prepare_template_host(t, td, st, labels);
  HostTables ht;
  build_tables(t, ht);
  if (!ctx->has_device) return ok();
  // every table in one device allocation, filled by one copy from a host
  // image (256-byte aligned parts; an empty table keeps a null pointer)
  struct Part { void** dst; const void* src; size_t bytes; size_t off; };
  auto part = [](auto** dst, const auto& v) {
    return Part{(void**)dst, (const void*)v.data(), v.size() * sizeof(v[0]), 0};
  };
  Part parts[] = {part(&t.d_codebook, t.codebook),   part(&t.d_frag_bf16, ht.frag_bf16),
                  part(&t.d_frag_f32, ht.frag_f32),  part(&t.d_cnorm, ht.cnorm),
                  part(&t.d_counts, ht.counts),      part(&t.d_counts16, ht.counts16),
                  part(&t.d_weights, t.weights),     part(&t.d_boxes, t.boxes),
                  part(&t.d_groups, t.groups),       part(&t.d_coef, t.coef),
                  part(&t.d_resp, ht.resp)};
  size_t total = 0;
  for (Part& q : parts) {
    q.off = total;
    total += (q.bytes + 255) & ~(size_t)255;
  }
  for (Part& q : parts) *q.dst = nullptr;
  if (total == 0) return ok();
  std::vector<char> image(total, 0);
  for (const Part& q : parts)
    if (q.bytes) std::memcpy(image.data() + q.off, q.src, q.bytes);
  char* blob = nullptr;
  HIP_TRY(hipMalloc((void**)&blob, total));
  t.d_blob = blob;
  HIP_TRY(hipMemcpy(blob, image.data(), total, hipMemcpyHostToDevice));
  for (const Part& q : parts)
    if (q.bytes) *q.dst = blob + q.off;
  return ok();
}

vqnnf_status check_template_map(const vqnnf_fmap* tmpl) {
  vqnnf_status s = check_map(tmpl, "template");
  if (s) return s;
  if (tmpl->dtype != VQNNF_F32 && tmpl->dtype != VQNNF_RGB8)
    return fail(VQNNF_EINVAL, "template: dtype must be VQNNF_F32 or VQNNF_RGB8");
  if (tmpl->H > 255 || tmpl->W > 255)
    return fail(VQNNF_EINVAL, "template: sides must be <= 255 (window histograms are 16-bit)");
  if (tmpl->dtype == VQNNF_RGB8) return ok();
  const int64_t np = (int64_t)tmpl->H * tmpl->W, st = tmpl->pixel_stride ? tmpl->pixel_stride : tmpl->D;
  const int D = tmpl->D;
  const float* base = (const float*)tmpl->data;
  // first pixel in [p0, p1) with an infinite or NaN value (all exponent bits
  // set), or -1
  auto scan = [&](int64_t p0, int64_t p1) -> int64_t {
    for (int64_t p = p0; p < p1; ++p) {
      const float* v = base + p * st;
      uint32_t bad = 0u;
      for (int d = 0; d < D; ++d) {
        uint32_t b;
        std::memcpy(&b, v + d, 4);
        bad |= (uint32_t)((b & 0x7f800000u) == 0x7f800000u);
      }
      if (bad) return p;
    }
    return -1;
  };
  int64_t first = -1;
  const unsigned hw = std::thread::hardware_concurrency();
  const int nt = np * D >= (int64_t)1 << 22 ? (int)std::min<unsigned>(8u, std::max(1u, hw)) : 1;
  if (nt == 1) {
    first = scan(0, np);
  } else {
    // large templates: contiguous pixel ranges on nt threads, the lowest hit wins
    std::vector<int64_t> hit(nt, -1);
    std::vector<std::thread> th;
    const int64_t per = (np + nt - 1) / nt;
    for (int i = 0; i < nt; ++i)
      th.emplace_back([&, i]() { hit[i] = scan(std::min(np, i * per), std::min(np, (i + 1) * per)); });
    for (std::thread& x : th) x.join();
    for (int i = 0; i < nt && first < 0; ++i) first = hit[i];
  }
  if (first >= 0) return fail(VQNNF_EINVAL, "template: non-finite value at pixel %lld", (long long)first);
  return ok();
}

vqnnf_status check_query(const vqnnf_ctx* c, const vqnnf_template* t, const vqnnf_fmap* q,
                         int prec) {
  vqnnf_status s = check_map(q, "query");
  if (s) return s;
  if (q->D != t->t.D) return fail(VQNNF_EINVAL, "query D=%d differs from template D=%d", q->D, t->t.D);
  if (prec != VQNNF_PREC_FP32_PLAIN && prec != VQNNF_PREC_BF16_REFINED && prec != VQNNF_PREC_FP8_REFINED)
    return fail(VQNNF_EINVAL, "unknown precision %d", prec);
  if (prec == VQNNF_PREC_FP8_REFINED && q->dtype != VQNNF_FP8_E4M3)
    return fail(VQNNF_EINVAL, "VQNNF_PREC_FP8_REFINED needs an FP8 E4M3 query map (got dtype %d)", q->dtype);
  (void)c;
  return ok();
}

// FP8 maps take the refined BF16 search (their codes are exact in BF16).
int32_t search_prec(int32_t prec) {
  return prec == VQNNF_PREC_FP8_REFINED ? VQNNF_PREC_BF16_REFINED : prec;
}

vqnnf_status need_device(const vqnnf_ctx* c) {
  if (!c->has_device)
    return fail(VQNNF_ENOTSUP, "context has no device (created with vqnnf_ctx_create_host)");
  return ok();
}

float unpack_score(unsigned long long key) {
  uint32_t o = (uint32_t)(key >> 32);
  uint32_t bits = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
  float f;
  std::memcpy(&f, &bits, 4);
  return f;
}

vqnnf_status read_best(vqnnf_ctx* c, int ow, int32_t* best_xy, float* best_score) {
  if (!best_xy && !best_score) return ok();
  unsigned long long key = 0;
  HIP_TRY(hipMemcpyAsync(&key, c->control.p, 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  uint32_t idx = 0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFu);
  if (best_xy) {
    best_xy[0] = (int32_t)(idx % (uint32_t)ow);
    best_xy[1] = (int32_t)(idx / (uint32_t)ow);
  }
  if (best_score) *best_score = unpack_score(key);
  return ok();
}

size_t mask_words(const DeviceTemplate& t) { return (size_t)(t.geom.kpad + 31) / 32; }

// Device scratch of one pair's path: by default the context's buffers;
// vqnnf_match_noalloc points them into its fixed array.
struct PairBufs {
  char* control;         // [0]: u64 best key, [8]: u32 worklist counter
  uint8_t* labels;       // [n_pix]
  uint32_t* wl_pix;      // [n_pix] re-score worklist
  uint32_t* wl_mask;     // [n_pix][mask_words] candidate masks
  void* partials;        // on-chip score partial sums
};
PairBufs ctx_bufs(const vqnnf_ctx* c) {
  return PairBufs{(char*)c->control.p, (uint8_t*)c->labels.p, (uint32_t*)c->wl_pix.p,
                  (uint32_t*)c->wl_mask.p, c->partials.p};
}

vqnnf_status save_tune_file(vqnnf_ctx* c);

// Shape class of a refined assignment for the schedule tuner: D, padded
// codebook size, storage, row alignment and the map size to a power of two.
std::vector<int> assign_key(const AssignArgs& a, int n_variants) {
  int lg = 0;
  while (lg < 40 && ((int64_t)1 << lg) < a.n_pix) ++lg;
  return {a.D, a.t->geom.kpad, a.dtype, n_variants, lg};
}

vqnnf_status run_assign(vqnnf_ctx* c, const vqnnf_template* tp, const vqnnf_fmap* q, int prec,
                        uint8_t* labels, bool counter_zeroed, const PairBufs& b, bool allow_tune = true) {
  const DeviceTemplate& t = tp->t;
  AssignArgs a{};
  a.q = q->data;
  a.stride = map_stride(q);
  a.img_w = q->W;
  a.img_h = q->H;
  a.n_pix = (int64_t)q->H * q->W;
  a.D = q->D;
  a.dtype = q->dtype;
  a.t = &t;
  a.labels = labels;
  const ScaledSet* ss = nullptr;
  if (q->dtype == VQNNF_FP8_E4M3) {
    for (const ScaledSet& x : t.scaled)
      if (std::memcmp(x.scale.data(), q->channel_scale, sizeof(float) * t.D) == 0) ss = &x;
    if (!ss) return fail(VQNNF_EINVAL, "FP8 tables were not prepared for this map");
  }
  a.frag_bf16 = ss ? ss->d_frag_bf16 : t.d_frag_bf16;
  a.frag_f32 = ss ? ss->d_frag_f32 : t.d_frag_f32;
  a.scale = ss ? ss->d_scale : nullptr;
  a.variant = c->assign_variant;
  const bool lowd = lowd_supported(q->dtype, q->D);
  if (prec == VQNNF_PREC_FP32_PLAIN) {
    if (lowd) HIP_TRY(launch_assign_lowd(a, false, c->stream));
    else HIP_TRY(launch_assign_plain(a, c->stream, c->n_cu));
    return ok();
  }
  a.wl_count = (uint32_t*)(b.control + 8);
  a.wl_pix = b.wl_pix;
  a.wl_mask = b.wl_mask;
  a.bound = ss ? ss->bound : (q->dtype == VQNNF_F32) ? t.bound_f32q : t.bound_bf16q;
  if (c->dbg_scores && !lowd) {
    if (a.n_pix * (int64_t)t.geom.kpad > c->dbg_cap)
      return fail(VQNNF_EINVAL, "debug score buffer holds %lld floats; this map needs %lld",
                  (long long)c->dbg_cap, (long long)(a.n_pix * t.geom.kpad));
    a.dump = c->dbg_scores;
  }
  bool launched = false;
  if (!lowd && !a.variant) {
    const int nv = refined_variants(a);
    const std::vector<int> key = assign_key(a, nv);
    auto it = c->avar_cache.find(key);
    if (it != c->avar_cache.end()) {
      a.variant = it->second;
    } else if (nv > 1 && c->autotune && !c->capturing && allow_tune) {
      // time every schedule twice on this very call (each run clears the
      // worklist counter and writes the same labels and worklist), keep the
      // fastest for the shape class; the last run's results stand
      set_timing_hook(nullptr);
      std::vector<hipEvent_t> ev(2 * nv);
      for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
      for (int rep = 0; rep < 2; ++rep)
        for (int v = 1; v <= nv; ++v) {
          a.variant = v;
          HIP_TRY(launch_fill_u32(a.wl_count, 0u, 1, c->stream));
          if (rep == 1) HIP_TRY(hipEventRecord(ev[2 * (v - 1)], c->stream));
          HIP_TRY(launch_assign_refined(a, c->stream, c->n_cu));
          if (rep == 1) HIP_TRY(hipEventRecord(ev[2 * (v - 1) + 1], c->stream));
        }
      HIP_TRY(hipEventSynchronize(ev.back()));
      float best_ms = 1e30f;
      int best = nv;
      for (int v = 1; v <= nv; ++v) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ev[2 * (v - 1)], ev[2 * (v - 1) + 1]));
        if (ms < best_ms) { best_ms = ms; best = v; }
      }
      for (auto& e : ev) hipEventDestroy(e);
      if (c->timing) {
        TimingHook h{hook_begin, hook_end, c};
        set_timing_hook(&h);
      }
      c->avar_cache[key] = best;
      vqnnf_status st = save_tune_file(c);
      if (st) return st;
      launched = true;
    }
  }
  if (!launched) {
    if (!counter_zeroed) HIP_TRY(launch_fill_u32(a.wl_count, 0u, 1, c->stream));
    if (lowd) HIP_TRY(launch_assign_lowd(a, true, c->stream));
    else HIP_TRY(launch_assign_refined(a, c->stream, c->n_cu));
  }
  HIP_TRY(launch_rescore(a, c->stream, c->n_cu));
  return ok();
}

vqnnf_status assign_scratch(vqnnf_ctx* c, const vqnnf_template* tp, int64_t n_pix, int prec,
                            bool own_labels) {
  size_t lab = own_labels ? (size_t)n_pix : 0;
  size_t wp = prec == VQNNF_PREC_BF16_REFINED ? (size_t)n_pix * 4 : 0;
  size_t wm = prec == VQNNF_PREC_BF16_REFINED ? (size_t)n_pix * 4 * mask_words(tp->t) : 0;
  vqnnf_status s = check_cap(c, {{&c->control, 64}, {&c->labels, lab}, {&c->wl_pix, wp},
                                 {&c->wl_mask, wm}});
  if (s) return s;
  if ((s = need_device(c))) return s;
  if ((s = ensure(c, c->control, 64, "control block"))) return s;
  if (own_labels && (s = ensure(c, c->labels, lab, "label map"))) return s;
  if (wp && (s = ensure(c, c->wl_pix, wp, "re-score worklist"))) return s;
  if (wm && (s = ensure(c, c->wl_mask, wm, "re-score candidate masks"))) return s;
  return ok();
}

vqnnf_status check_score_dims(const vqnnf_template* tp, int H, int W) {
  const DeviceTemplate& t = tp->t;
  if (H < 1 || W < 1) return fail(VQNNF_EINVAL, "H and W must be >= 1");
  if ((int64_t)H * W >= (1ll << 31)) return fail(VQNNF_EINVAL, "H*W must be < 2^31");
  if (t.w > W || t.h > H)
    return fail(VQNNF_EINVAL, "template %dx%d larger than the %dx%d map", t.w, t.h, W, H);
  if (t.weighted) {
    // the bank kernel addresses a band of h + 66 integral-image rows with
    // 32-bit byte offsets
    const int64_t row_bytes = (int64_t)(W + 1) * t.k * 4;
    if ((int64_t)(t.h + 66) * row_bytes >= (1ll << 32))
      return fail(VQNNF_ENOTSUP, "weighted bank: a %d-column map with k = %d is too wide for the bank kernel",
                  W, t.k);
  }
  return ok();
}

// partials: the on-chip score's partial sums (null: the context's buffer).
// tune: the first call on a new shape may time tile heights (allocates
// events); false uses the tuned height if known, else the default sizing.
vqnnf_status enqueue_score(vqnnf_ctx* c, const vqnnf_template* t, const uint8_t* labels,
                                  const int32_t* P, int32_t H, int32_t W, float* heatmap,
                                  unsigned long long* best, bool zeroed,
                                  const uint16_t* P16 = nullptr, void* partials = nullptr,
                                  bool tune = true) {
  ScoreArgs a{};
  a.t = &t->t;
  a.labels = labels;
  a.P = P;
  a.P16 = P16;
  a.H = H;
  a.W = W;
  a.heatmap = heatmap;
  a.best = best;
  a.partials = partials ? partials : c->partials.p;
  a.n_cu = c->n_cu;
  if (!zeroed) HIP_TRY(launch_zero_u64(a.best, c->stream));
  if (labels) {
    size_t lds = 0;
    const DeviceTemplate& d = t->t;
    bool uni = true;
    for (int f = 2; f < d.n_filters; ++f) uni = uni && d.weights[f] == d.weights[1];
    const std::vector<int> key = {d.w, d.h, d.grid.g, d.geom.kpad, H, W, uni ? 1 : 0};
    // a tile choice: window rows per tile, plus kScoreWide for 32-channel
    // blocks (untuned: the default block width and height)
    auto set_choice = [&](int v) {
      a.tyw = v & (kScoreWide - 1);
      a.kgsel = (v & kScoreWide) ? 2 : 1;
    };
    auto it = c->tyw_cache.find(key);
    if (it != c->tyw_cache.end()) {
      set_choice(it->second);
    } else if (tune && c->autotune && !c->capturing) {
      // time each candidate block width and tile height twice on this very
      // call (every run writes the same heatmap and key), keep the fastest
      // for the shape
      const int oh = H - d.h + 1;
      std::vector<int> cand;
      int def = 0;
      for (int wide : {0, 1}) {
        if (wide && !fused_wide_allowed(d)) continue;
        const int flag = wide ? kScoreWide : 0;
        const int dv = fused_default_tyw(d, H, W, c->n_cu, wide != 0) | flag;
        if ((wide != 0) == fused_default_wide(d)) def = dv;
        cand.push_back(dv);
        for (int v : {16, 32, 64, 128, 256})
          if (v <= oh && std::find(cand.begin(), cand.end(), v | flag) == cand.end()) cand.push_back(v | flag);
      }
      set_timing_hook(nullptr);
      std::vector<hipEvent_t> ev(2 * cand.size());
      for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
      for (int rep = 0; rep < 2; ++rep)
        for (size_t ci = 0; ci < cand.size(); ++ci) {
          set_choice(cand[ci]);
          if (rep == 1) HIP_TRY(hipEventRecord(ev[2 * ci], c->stream));
          HIP_TRY(launch_score_fused(a, c->stream, &lds));
          if (rep == 1) HIP_TRY(hipEventRecord(ev[2 * ci + 1], c->stream));
        }
      HIP_TRY(hipEventSynchronize(ev.back()));
      float best_ms = 1e30f;
      int best = def;
      for (size_t ci = 0; ci < cand.size(); ++ci) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ev[2 * ci], ev[2 * ci + 1]));
        if (ms < best_ms) { best_ms = ms; best = cand[ci]; }
      }
      for (auto& e : ev) hipEventDestroy(e);
      if (c->timing) {
        TimingHook h{hook_begin, hook_end, c};
        set_timing_hook(&h);
      }
      c->tyw_cache[key] = best;
      vqnnf_status st = save_tune_file(c);
      if (st) return st;
      return ok();   // the last candidate's run already produced the result
    }
    HIP_TRY(launch_score_fused(a, c->stream, &lds));
  } else if (t->t.weighted) {
    HIP_TRY(launch_score_bank(a, c->stream));
  } else {
    HIP_TRY(launch_score_integral(a, c->stream));
  }
  return ok();
}

// Channels of the matching path's integral image: weighted banks read it
// mod 2^16 in channel pairs, so their channel count is rounded up to even.
int int_channels(const DeviceTemplate& d) { return d.weighted ? d.k + (d.k & 1) : d.k; }

// Score of one pair from a label map: the on-chip kernel, or the integral
// image and the integral score for banks the on-chip kernel does not take.
vqnnf_status enqueue_score_labels(vqnnf_ctx* c, const vqnnf_template* t, const uint8_t* lab, int H,
                                  int W, float* heatmap, unsigned long long* key) {
  if (fused_supported(t->t)) return enqueue_score(c, t, lab, nullptr, H, W, heatmap, key, true);
  const int k = int_channels(t->t);
  const int64_t R = (H + kIntTile - 1) / kIntTile, S = (W + kIntTile - 1) / kIntTile;
  IntegralArgs a{};
  a.labels = lab;
  a.H = H;
  a.W = W;
  a.k = k;
  // weighted banks: P mod 2^16 with an even channel count (pad channel empty)
  if (t->t.weighted) a.P16 = (uint16_t*)c->int_p.p;
  else a.P = (int32_t*)c->int_p.p;
  a.rsh = (int32_t*)c->int_side.p;
  a.cbh = a.rsh + (size_t)H * S * k;
  a.th = a.cbh + (size_t)R * W * k;
  HIP_TRY(launch_integral(a, c->stream));
  return enqueue_score(c, t, nullptr, a.P, H, W, heatmap, key, true, a.P16);
}

// Scratch for matching the given pairs one after another (sized for the largest).
vqnnf_status pair_scratch(vqnnf_ctx* c, const vqnnf_template* const* t, const vqnnf_fmap* const* q,
                          int n, int prec, size_t control) {
  size_t lab = 0, wp = 0, wm = 0, side = 0, pbytes = 0, partb = 0;
  for (int i = 0; i < n; ++i) {
    const int64_t np = (int64_t)q[i]->H * q[i]->W;
    const DeviceTemplate& d = t[i]->t;
    lab = std::max(lab, (size_t)np);
    if (prec == VQNNF_PREC_BF16_REFINED) {
      wp = std::max(wp, (size_t)np * 4);
      wm = std::max(wm, (size_t)np * 4 * mask_words(d));
    }
    if (fused_supported(d)) {
      partb = std::max(partb, fused_partial_bytes(d, q[i]->H, q[i]->W));
    } else {
      const int64_t R = (q[i]->H + kIntTile - 1) / kIntTile, S = (q[i]->W + kIntTile - 1) / kIntTile;
      const int kc = int_channels(d);
      side = std::max(side, (size_t)((int64_t)q[i]->H * S + R * q[i]->W + R * S) * kc * 4);
      pbytes = std::max(pbytes, (size_t)(q[i]->H + 1) * (q[i]->W + 1) * kc * (d.weighted ? 2 : 4));
    }
  }
  vqnnf_status s = check_cap(c, {{&c->control, control}, {&c->labels, lab}, {&c->wl_pix, wp},
                                 {&c->wl_mask, wm}, {&c->int_side, side}, {&c->int_p, pbytes},
                                 {&c->partials, partb}});
  if (s) return s;
  if ((s = need_device(c))) return s;
  if ((s = ensure(c, c->control, control, "control block"))) return s;
  if ((s = ensure(c, c->labels, lab, "label map"))) return s;
  if (wp && (s = ensure(c, c->wl_pix, wp, "re-score worklist"))) return s;
  if (wm && (s = ensure(c, c->wl_mask, wm, "re-score candidate masks"))) return s;
  if (partb && (s = ensure(c, c->partials, partb, "score partial sums"))) return s;
  if (side && (s = ensure(c, c->int_side, side, "integral-image side arrays"))) return s;
  if (pbytes && (s = ensure(c, c->int_p, pbytes, "integral image"))) return s;
  return ok();
}

// Enqueues the whole path of one pair on the context stream: assignment
// (+ re-score), then the on-chip score, or the integral image and the
// integral score for banks the on-chip kernel does not take.  The best key
// must be zero; the worklist counter is cleared here unless the caller did.
vqnnf_status enqueue_pair(vqnnf_ctx* c, const vqnnf_template* t, const vqnnf_fmap* q, int prec,
                          float* heatmap, unsigned long long* key, bool counter_zeroed) {
  uint8_t* lab = (uint8_t*)c->labels.p;
  vqnnf_status s = run_assign(c, t, q, prec, lab, counter_zeroed, ctx_bufs(c));
  if (s) return s;
  return enqueue_score_labels(c, t, lab, q->H, q->W, heatmap, key);
}

// Writes every tuning result of the context to its tune file (if any):
// written to a temporary file and renamed, so a reader never sees half a file.
vqnnf_status save_tune_file(vqnnf_ctx* c) {
  if (c->tune_file.empty()) return ok();
  const std::string tmp = c->tune_file + ".tmp" + std::to_string((long long)(uintptr_t)c);
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return fail(VQNNF_EINVAL, "cannot write the tune file %s", tmp.c_str());
  auto put = [&](char kind, const std::map<std::vector<int>, int>& m) {
    for (const auto& e : m) {
      std::fprintf(f, "%c %d", kind, c->n_cu);
      for (int x : e.first) std::fprintf(f, " %d", x);
      std::fprintf(f, " %d\n", e.second);
    }
  };
  put('a', c->avar_cache);
  put('s', c->tyw_cache);
  put('b', c->btyw_cache);
  const bool bad = std::fclose(f) != 0;
  if (bad || std::rename(tmp.c_str(), c->tune_file.c_str()) != 0) {
    std::remove(tmp.c_str());
    return fail(VQNNF_EINVAL, "cannot write the tune file %s", c->tune_file.c_str());
  }
  return ok();
}

// Byte layout of vqnnf_match_noalloc's fixed scratch for one pair: the
// control block, the label map, the worklist and masks (refined path) and
// the score partials, each part 256-byte aligned.
struct NoAllocLayout {
  size_t labels, wl_pix, wl_mask, partials, total;
};
NoAllocLayout noalloc_layout(const DeviceTemplate& t, int H, int W, int prec) {
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t np = (size_t)H * W;
  const bool refined = prec == VQNNF_PREC_BF16_REFINED;
  NoAllocLayout l{};
  l.labels = 256;
  l.wl_pix = l.labels + al(np);
  l.wl_mask = l.wl_pix + (refined ? al(np * 4) : 0);
  l.partials = l.wl_mask + (refined ? al(np * 4 * mask_words(t)) : 0);
  l.total = l.partials + al(fused_partial_bytes(t, H, W));
  return l;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

const char* vqnnf_last_error(void) { return g_err.c_str(); }
const char* vqnnf_version(void) { return "vqnnf-gfx950 0.1"; }

vqnnf_status vqnnf_ctx_create(void* hip_stream, uint64_t scratch_cap_bytes, vqnnf_ctx** out) {
  if (!out) return fail(VQNNF_EINVAL, "null output pointer");
  *out = nullptr;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(VQNNF_ENOTSUP, "device %d is %s; this library is built for gfx950", dev, prop.gcnArchName);
  // the fixed scratch of vqnnf_match_noalloc, resolved once per device
  HIP_TRY(noalloc_scratch_init(dev));
  auto* c = new vqnnf_ctx();
  c->has_device = true;
  c->device = dev;
  c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  c->stream = (hipStream_t)hip_stream;
  c->cap = scratch_cap_bytes ? scratch_cap_bytes : (16ull << 30);
  if (const char* v = std::getenv("VQNNF_ASSIGN_VARIANT")) c->assign_variant = std::atoi(v);
  *out = c;
  return ok();
}

vqnnf_status vqnnf_ctx_create_host(uint64_t scratch_cap_bytes, vqnnf_ctx** out) {
  if (!out) return fail(VQNNF_EINVAL, "null output pointer");
  auto* c = new vqnnf_ctx();
  c->has_device = false;
  c->cap = scratch_cap_bytes ? scratch_cap_bytes : (16ull << 30);
  *out = c;
  return ok();
}

void vqnnf_ctx_destroy(vqnnf_ctx* c) {
  if (!c || c->magic != kCtxMagic) return;
  if (c->has_device) {
    hipStreamSynchronize(c->stream);
    if (c->gexec) hipGraphExecDestroy(c->gexec);
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    Buffer* bs[] = {&c->control, &c->labels, &c->wl_pix, &c->wl_mask, &c->int_side, &c->int_p,
                    &c->partials, &c->keys, &c->pca, &c->m_labels, &c->m_count, &c->m_wl_pix, &c->m_wl_mask,
                    &c->b_part, &c->b_tab};
    for (Buffer* b : bs)
      if (b->p) hipFree(b->p);
    for (auto& mp : c->mplans)
      for (Buffer* b : {&mp.frag, &mp.cnorm, &mp.passes, &mp.outs})
        if (b->p) hipFree(b->p);
    for (auto& r : c->pending) { hipEventDestroy(r.a); hipEventDestroy(r.b); }
    for (auto e : c->pool) hipEventDestroy(e);
  }
  c->magic = 0;
  delete c;
}

// k-means of several templates on the device in one set of launches:
// codebooks (FP32) and the templates' NNFs, bit-identical to kmeans_host +
// assign_host.  Temporary device memory, released before returning.
static vqnnf_status kmeans_device(vqnnf_ctx* c, const std::vector<vqnnf_template*>& tps,
                                  const vqnnf_fmap* const* tmpls, int iters, const uint64_t* seeds,
                                  std::vector<std::vector<uint8_t>>& labels) {
  const size_t n = tps.size();
  std::vector<size_t> off(n + 1, 0);
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  struct Sz { size_t x, xt, c, c32, lab, idx, start, d2, state, pdist, pidx; };
  std::vector<Sz> sz(n);
  for (size_t i = 0; i < n; ++i) {
    const DeviceTemplate& t = tps[i]->t;
    const size_t l = (size_t)t.w * t.h, kd = (size_t)t.k * t.D, nch = (t.k + 15) / 16;
    sz[i] = {al(l * t.D * 4), al(l * t.D * 4), al(kd * 8), al(kd * 4), al(l), al(l * 4), al((t.k + 1) * 4), al(l * 8), al(8),
             al(nch * l * 8), al(nch * l)};
    const Sz& z = sz[i];
    off[i + 1] = off[i] + z.x + z.xt + z.c + z.c32 + z.lab + z.idx + z.start + z.d2 + z.state + z.pdist + z.pidx;
  }
  const size_t jobs_off = al(off[n]);
  const size_t total = jobs_off + al(n * sizeof(KmJob));
  if (total > c->cap) return fail(VQNNF_ENOMEM, "k-means needs %zu bytes of device memory, cap %llu", total,
                                  (unsigned long long)c->cap);
  char* arena = nullptr;
  HIP_TRY(hipMalloc((void**)&arena, total));
  std::vector<KmJob> jobs(n);
  std::vector<std::vector<float>> packed(n);    // strided maps, packed (alive until the sync)
  hipError_t e = hipSuccess;
  for (size_t i = 0; i < n && e == hipSuccess; ++i) {
    const DeviceTemplate& t = tps[i]->t;
    const Sz& z = sz[i];
    char* b = arena + off[i];
    KmJob& j = jobs[i];
    j.x = (const float*)b; b += z.x;
    j.xt = (float*)b; b += z.xt;
    j.c = (double*)b; b += z.c;
    j.c32 = (float*)b; b += z.c32;
    j.lab = (uint8_t*)b; b += z.lab;
    j.idx = (int*)b; b += z.idx;
    j.start = (int*)b; b += z.start;
    j.d2 = (double*)b; b += z.d2;
    j.state = (uint64_t*)b; b += z.state;
    j.pdist = (double*)b; b += z.pdist;
    j.pidx = (uint8_t*)b;
    j.seed = seeds[i];
    j.l = t.w * t.h;
    j.D = t.D;
    j.k = t.k;
    const vqnnf_fmap* m = tmpls[i];
    const int64_t st = m->pixel_stride ? m->pixel_stride : m->D;
    const float* src = (const float*)m->data;
    if (st != t.D) {   // one contiguous copy instead of one per pixel
      packed[i].resize((size_t)j.l * t.D);
      for (int64_t q = 0; q < j.l; ++q)
        std::memcpy(&packed[i][(size_t)q * t.D], src + q * st, (size_t)t.D * 4);
      src = packed[i].data();
    }
    e = hipMemcpyAsync((void*)j.x, src, (size_t)j.l * t.D * 4, hipMemcpyHostToDevice, c->stream);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(arena + jobs_off, jobs.data(), n * sizeof(KmJob), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = launch_kmeans((const KmJob*)(arena + jobs_off), jobs, iters, c->stream);
  labels.assign(n, {});
  for (size_t i = 0; i < n && e == hipSuccess; ++i) {
    DeviceTemplate& t = tps[i]->t;
    t.codebook.resize((size_t)t.k * t.D);
    labels[i].resize((size_t)jobs[i].l);
    e = hipMemcpyAsync(t.codebook.data(), jobs[i].c32, t.codebook.size() * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(labels[i].data(), jobs[i].lab, labels[i].size(), hipMemcpyDeviceToHost, c->stream);
  }
  const hipError_t e2 = hipStreamSynchronize(c->stream);
  hipFree(arena);
  if (e == hipSuccess) e = e2;
  if (e != hipSuccess) return fail(VQNNF_EHIP, "k-means on the device: %s", hipGetErrorString(e));
  return ok();
}

static vqnnf_status new_template(vqnnf_ctx* ctx, const vqnnf_fmap* tmpl, int32_t k, int32_t iters,
                                 const vqnnf_filter_desc* bank, int32_t n_desc, vqnnf_template** out) {
  vqnnf_status s;
  if ((s = check_template_map(tmpl))) return s;
  if (k < 1 || k > kMaxK) return fail(VQNNF_EINVAL, "k=%d outside [1, %d]", k, kMaxK);
  if (iters < 0) return fail(VQNNF_EINVAL, "lloyd_iters must be >= 0");
  auto* tp = new vqnnf_template();
  tp->ctx = ctx;
  DeviceTemplate& t = tp->t;
  t.w = tmpl->W;
  t.h = tmpl->H;
  t.D = tmpl->D;
  t.k = k;
  if ((s = expand_bank(bank, n_desc, t.w, t.h, t))) { delete tp; return s; }
  *out = tp;
  return ok();
}

// An RGB template as its FP32 colour features (the map `f` points at `buf`).
static vqnnf_status rgb_template_features(const vqnnf_fmap* m, std::vector<float>& buf, vqnnf_fmap& f) {
  vqnnf_status s = check_template_map(m);
  if (s) return s;
  buf.resize((size_t)m->H * m->W * 27);
  rgb_patch_features_host((const uint8_t*)m->data, m->H, m->W, map_stride(m), buf.data());
  f = *m;
  f.data = buf.data();
  f.dtype = VQNNF_F32;
  f.D = 27;
  f.pixel_stride = 27;
  f.channel_scale = nullptr;
  return ok();
}

static vqnnf_status make_template(vqnnf_ctx* ctx, const vqnnf_fmap* tmpl, const float* codebook,
                                  int32_t k, int32_t iters, uint64_t seed,
                                  const vqnnf_filter_desc* bank, int32_t n_desc,
                                  vqnnf_template** out) {
  vqnnf_status s;
  if (!out) return fail(VQNNF_EINVAL, "null output pointer");
  *out = nullptr;
  if ((s = check_ctx(ctx))) return s;
  std::vector<float> rgb_buf;
  vqnnf_fmap rgb_f{};
  if (tmpl && tmpl->dtype == VQNNF_RGB8) {
    if ((s = rgb_template_features(tmpl, rgb_buf, rgb_f))) return s;
    tmpl = &rgb_f;
  }
  vqnnf_template* tp = nullptr;
  if ((s = new_template(ctx, tmpl, k, iters, bank, n_desc, &tp))) return s;
  DeviceTemplate& t = tp->t;
  int64_t n = (int64_t)t.w * t.h;
  int64_t st = tmpl->pixel_stride ? tmpl->pixel_stride : tmpl->D;
  const float* td = (const float*)tmpl->data;
  std::vector<std::vector<uint8_t>> lab;
  if (codebook) {
    for (int64_t i = 0; i < (int64_t)k * t.D; ++i)
      if (!std::isfinite(codebook[i])) { delete tp; return fail(VQNNF_EINVAL, "codebook: non-finite value"); }
    t.codebook.assign(codebook, codebook + (size_t)k * t.D);
  } else if (ctx->has_device) {
    std::vector<vqnnf_template*> one{tp};
    if ((s = kmeans_device(ctx, one, &tmpl, iters, &seed, lab))) { delete tp; return s; }
  } else {
    std::vector<double> x((size_t)n * t.D);
    for (int64_t p = 0; p < n; ++p)
      for (int d = 0; d < t.D; ++d) x[(size_t)p * t.D + d] = (double)td[p * st + d];
    std::vector<double> c = kmeans_host(x, n, t.D, k, iters, seed);
    t.codebook.resize(c.size());
    for (size_t i = 0; i < c.size(); ++i) t.codebook[i] = (float)c[i];
  }
  if ((s = finish_template(ctx, tp, tmpl, lab.empty() ? nullptr : lab[0].data()))) {
    free_device(t);
    delete tp;
    return s;
  }
  *out = tp;
  return ok();
}

vqnnf_status vqnnf_codebook(vqnnf_ctx* ctx, const vqnnf_fmap* tmpl, int32_t k, int32_t lloyd_iters,
                            uint64_t seed, const vqnnf_filter_desc* bank, int32_t n_desc,
                            vqnnf_template** out) {
  return make_template(ctx, tmpl, nullptr, k, lloyd_iters, seed, bank, n_desc, out);
}

vqnnf_status vqnnf_codebook_batched(vqnnf_ctx* ctx, int32_t n, const vqnnf_fmap* const* tmpls,
                                    const int32_t* ks, int32_t lloyd_iters, const uint64_t* seeds,
                                    const vqnnf_filter_desc* const* banks, const int32_t* n_descs,
                                    vqnnf_template** out) {
  vqnnf_status s;
  if ((s = check_ctx(ctx))) return s;
  if (n < 1 || !tmpls || !ks || !seeds || !banks || !n_descs || !out)
    return fail(VQNNF_EINVAL, "batched codebooks: need n >= 1 and non-null arrays");
  for (int i = 0; i < n; ++i) out[i] = nullptr;
  // RGB templates as their FP32 colour features
  std::vector<std::vector<float>> rgb_buf(n);
  std::vector<vqnnf_fmap> rgb_f(n);
  std::vector<const vqnnf_fmap*> maps(tmpls, tmpls + n);
  for (int i = 0; i < n; ++i)
    if (tmpls[i] && tmpls[i]->dtype == VQNNF_RGB8) {
      if ((s = rgb_template_features(tmpls[i], rgb_buf[i], rgb_f[i]))) {
        const std::string msg = vqnnf_last_error();
        return fail(s, "template %d: %s", i, msg.c_str());
      }
      maps[i] = &rgb_f[i];
    }
  tmpls = maps.data();
  std::vector<vqnnf_template*> tps;
  auto drop = [&]() {
    for (vqnnf_template* tp : tps) {
      free_device(tp->t);
      delete tp;
    }
  };
  for (int i = 0; i < n; ++i) {
    vqnnf_template* tp = nullptr;
    if ((s = new_template(ctx, tmpls[i], ks[i], lloyd_iters, banks[i], n_descs[i], &tp))) {
      const std::string msg = vqnnf_last_error();
      drop();
      return fail(s, "template %d: %s", i, msg.c_str());
    }
    tps.push_back(tp);
  }
  std::vector<std::vector<uint8_t>> lab;
  if (ctx->has_device) {
    if ((s = kmeans_device(ctx, tps, tmpls, lloyd_iters, seeds, lab))) { drop(); return s; }
  } else {
    for (int i = 0; i < n; ++i) {
      DeviceTemplate& t = tps[i]->t;
      const int64_t np = (int64_t)t.w * t.h;
      const int64_t st = tmpls[i]->pixel_stride ? tmpls[i]->pixel_stride : tmpls[i]->D;
      const float* td = (const float*)tmpls[i]->data;
      std::vector<double> x((size_t)np * t.D);
      for (int64_t p = 0; p < np; ++p)
        for (int d = 0; d < t.D; ++d) x[(size_t)p * t.D + d] = (double)td[p * st + d];
      std::vector<double> c = kmeans_host(x, np, t.D, t.k, lloyd_iters, seeds[i]);
      t.codebook.resize(c.size());
      for (size_t q = 0; q < c.size(); ++q) t.codebook[q] = (float)c[q];
    }
  }
  for (int i = 0; i < n; ++i)
    if ((s = finish_template(ctx, tps[i], tmpls[i], lab.empty() ? nullptr : lab[i].data()))) {
      drop();
      return s;
    }
  for (int i = 0; i < n; ++i) out[i] = tps[i];
  return ok();
}

vqnnf_status vqnnf_pca_fit(const vqnnf_fmap* tmpl, int32_t d, float* mean, float* basis, float* variances) {
  vqnnf_status s;
  if (!tmpl || !mean || !basis) return fail(VQNNF_EINVAL, "null template or output pointer");
  std::vector<float> rgb_buf;
  vqnnf_fmap rgb_f{};
  if (tmpl->dtype == VQNNF_RGB8) {
    if ((s = rgb_template_features(tmpl, rgb_buf, rgb_f))) return s;
    tmpl = &rgb_f;
  } else if ((s = check_template_map(tmpl))) {
    return s;
  }
  if (d < 1 || d > std::min(tmpl->D, 64))
    return fail(VQNNF_EINVAL, "d=%d outside [1, min(D, 64)] (D = %d)", d, tmpl->D);
  std::vector<double> m, b, v;
  pca_fit_host((const float*)tmpl->data, (int64_t)tmpl->H * tmpl->W, map_stride(tmpl), tmpl->D, d, m, b, v);
  for (int t = 0; t < tmpl->D; ++t) mean[t] = (float)m[t];
  for (size_t i = 0; i < b.size(); ++i) basis[i] = (float)b[i];
  if (variances)
    for (int i = 0; i < d; ++i) variances[i] = (float)v[i];
  return ok();
}

vqnnf_status vqnnf_pca_project(vqnnf_ctx* c, const vqnnf_fmap* map, const float* mean, const float* basis,
                               int32_t d, float* out) {
  vqnnf_status s;
  if ((s = check_ctx(c))) return s;
  if ((s = check_map(map, "map"))) return s;
  if (!mean || !basis || !out) return fail(VQNNF_EINVAL, "null mean, basis or output");
  const int D = map->D;
  if (d < 1 || d > std::min(D, 64)) return fail(VQNNF_EINVAL, "d=%d outside [1, min(D, 64)] (D = %d)", d, D);
  for (int i = 0; i < d * D; ++i)
    if (!std::isfinite(basis[i])) return fail(VQNNF_EINVAL, "basis: non-finite value");
  for (int i = 0; i < D; ++i)
    if (!std::isfinite(mean[i])) return fail(VQNNF_EINVAL, "mean: non-finite value");
  // BF16 maps with aligned rows of whole 32-element groups: matrix cores, the
  // basis split into three BF16 terms (exact for every finite FP32 value it
  // is checked for), the centring applied as mean . basis
  const int64_t st = map_stride(map);
  bool mfma = map->dtype == VQNNF_BF16 && D % 32 == 0 && (uintptr_t)map->data % 16 == 0 && (st * 2) % 16 == 0 &&
              pca_mfma_lds(D, d) <= 160 * 1024;
  const int rbn = (d + 15) / 16, steps = D / 32;
  std::vector<uint16_t> frag;
  std::vector<float> mb;
  if (mfma) {
    frag.assign((size_t)steps * 3 * rbn * 64 * 8, 0);
    for (int i = 0; i < d && mfma; ++i)
      for (int t = 0; t < D; ++t) {
        const float b = basis[(size_t)i * D + t];
        const float h = bf16_round(b), r1 = b - h, l = bf16_round(r1), r2 = r1 - l, l2 = bf16_round(r2);
        if ((double)h + (double)l + (double)l2 != (double)b) { mfma = false; break; }
        const float terms[3] = {h, l, l2};
        const int s2 = t / 32, lg = (t % 32) / 8, e = t % 8, rb = i / 16, lane = (i % 16) + 16 * lg;
        for (int term = 0; term < 3; ++term)
          frag[((((size_t)s2 * 3 + term) * rbn + rb) * 64 + lane) * 8 + e] = bf16_bits(terms[term]);
      }
    mb.resize(d);
    for (int i = 0; i < d; ++i) {
      double acc = 0.0;
      for (int t = 0; t < D; ++t) acc += (double)mean[t] * (double)basis[(size_t)i * D + t];
      mb[i] = (float)acc;
    }
  }
  const size_t tb = mfma ? frag.size() * 2 + (size_t)d * 4 + 256 : ((size_t)d * D + 2 * (size_t)D) * sizeof(float);
  if ((s = check_cap(c, {{&c->pca, tb}}))) return s;
  if ((s = need_device(c))) return s;
  if ((s = ensure(c, c->pca, tb, "projection tables"))) return s;
  if (mfma) {
    uint4* dfrag = (uint4*)c->pca.p;
    float* dmb = (float*)((char*)c->pca.p + frag.size() * 2);
    HIP_TRY(hipMemcpyAsync(dfrag, frag.data(), frag.size() * 2, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(dmb, mb.data(), (size_t)d * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));   // host tables are released on return
    HookScope hs(c);
    HIP_TRY(launch_pca_mfma((const uint16_t*)map->data, st, map->H, map->W, D, dfrag, dmb, d, out, c->n_cu,
                            c->stream));
    return ok();
  }
  float* db = (float*)c->pca.p;
  float* dm = db + (size_t)d * D;
  float* ds = dm + D;
  std::vector<float> bt((size_t)d * D);      // t-major: the d values of element t together
  for (int i = 0; i < d; ++i)
    for (int t = 0; t < D; ++t) bt[(size_t)t * d + i] = basis[(size_t)i * D + t];
  HIP_TRY(hipMemcpyAsync(db, bt.data(), (size_t)d * D * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));   // the host copy of the table is released on return
  HIP_TRY(hipMemcpyAsync(dm, mean, (size_t)D * 4, hipMemcpyHostToDevice, c->stream));
  if (map->dtype == VQNNF_FP8_E4M3)
    HIP_TRY(hipMemcpyAsync(ds, map->channel_scale, (size_t)D * 4, hipMemcpyHostToDevice, c->stream));
  HookScope hs(c);
  HIP_TRY(launch_pca_project(map->data, map->dtype, map_stride(map), map->H, map->W, D,
                             map->dtype == VQNNF_FP8_E4M3 ? ds : nullptr, dm, db, d, out, c->stream));
  return ok();
}

vqnnf_status vqnnf_template_from_codebook(vqnnf_ctx* ctx, const vqnnf_fmap* tmpl,
                                          const float* codebook, int32_t k,
                                          const vqnnf_filter_desc* bank, int32_t n_desc,
                                          vqnnf_template** out) {
  if (!codebook) return fail(VQNNF_EINVAL, "null codebook");
  return make_template(ctx, tmpl, codebook, k, 0, 0, bank, n_desc, out);
}

void vqnnf_template_free(vqnnf_template* t) {
  if (!t || t->magic != kTplMagic) return;
  if (t->ctx && t->ctx->has_device) {
    hipStreamSynchronize(t->ctx->stream);
    free_device(t->t);
  }
  t->magic = 0;
  delete t;
}

vqnnf_status vqnnf_template_info(const vqnnf_template* t, int32_t* w, int32_t* h, int32_t* D,
                                 int32_t* k, int32_t* n_filters) {
  vqnnf_status s = check_tpl(nullptr, t);
  if (s) return s;
  if (w) *w = t->t.w;
  if (h) *h = t->t.h;
  if (D) *D = t->t.D;
  if (k) *k = t->t.k;
  if (n_filters) *n_filters = t->t.n_filters;
  return ok();
}

vqnnf_status vqnnf_template_codebook(const vqnnf_template* t, float* out) {
  vqnnf_status s = check_tpl(nullptr, t);
  if (s) return s;
  if (!out) return fail(VQNNF_EINVAL, "null output");
  std::memcpy(out, t->t.codebook.data(), t->t.codebook.size() * sizeof(float));
  return ok();
}

vqnnf_status vqnnf_template_labels(const vqnnf_template* t, uint8_t* out) {
  vqnnf_status s = check_tpl(nullptr, t);
  if (s) return s;
  if (!out) return fail(VQNNF_EINVAL, "null output");
  std::memcpy(out, t->t.labels.data(), t->t.labels.size());
  return ok();
}

vqnnf_status vqnnf_template_counts(const vqnnf_template* t, int32_t* out) {
  vqnnf_status s = check_tpl(nullptr, t);
  if (s) return s;
  if (!out) return fail(VQNNF_EINVAL, "null output");
  if (t->t.weighted)
    return fail(VQNNF_ENOTSUP, "the bank has weighted filters: use vqnnf_template_responses");
  std::memcpy(out, t->t.counts.data(), t->t.counts.size() * sizeof(int32_t));
  return ok();
}

vqnnf_status vqnnf_template_responses(const vqnnf_template* t, float* out) {
  vqnnf_status s = check_tpl(nullptr, t);
  if (s) return s;
  if (!out) return fail(VQNNF_EINVAL, "null output");
  const DeviceTemplate& d = t->t;
  if (d.weighted) {
    std::memcpy(out, d.resp.data(), d.resp.size() * sizeof(float));
  } else {
    for (size_t i = 0; i < d.counts.size(); ++i) out[i] = (float)d.counts[i];
  }
  return ok();
}

vqnnf_status vqnnf_paper_bank(int32_t w, int32_t h, int32_t filter_set, int32_t n_scales,
                              vqnnf_filter_desc* out, float* bin_weights, int32_t capacity,
                              int32_t* n_out) {
  enum { GAUSS, HAAR2X, HAAR2Y, HAAR3X, HAAR3Y };
  static const int kMembers[4][5] = {{GAUSS}, {GAUSS, HAAR2X, HAAR2Y}, {GAUSS, HAAR3X, HAAR3Y},
                                     {GAUSS, HAAR2X, HAAR2Y, HAAR3X, HAAR3Y}};
  static const int kSize[4] = {1, 3, 3, 5};
  if (!out || !bin_weights || !n_out) return fail(VQNNF_EINVAL, "null output pointer");
  if (filter_set < VQNNF_BANK_GAUSS || filter_set > VQNNF_BANK_23RECT)
    return fail(VQNNF_EINVAL, "unknown filter set %d", filter_set);
  if (n_scales < 1) return fail(VQNNF_EINVAL, "n_scales must be >= 1 (got %d)", n_scales);
  if (w < 1 || h < 1) return fail(VQNNF_EINVAL, "template sides must be >= 1");
  const int per = kSize[filter_set];
  if ((int64_t)n_scales * per > capacity)
    return fail(VQNNF_EINVAL, "capacity %d < %d descs", capacity, n_scales * per);
  for (int sc = 1; sc <= n_scales; ++sc)
    if (w / sc < 3 || h / sc < 3)
      return fail(VQNNF_EINVAL, "scale %d: the %dx%d sub-window has empty 3x3 bins", sc, w / sc, h / sc);
  // 3x3 coarse Gaussian, sigma 2, centre 1; Haar factors per column (x) or row (y)
  double g[3][3];
  for (int b = 0; b < 3; ++b)
    for (int a = 0; a < 3; ++a) g[b][a] = std::exp(-(double)((a - 1) * (a - 1) + (b - 1) * (b - 1)) / 8.0);
  static const double kF2[3] = {1.0, 0.0, -1.0}, kF3[3] = {1.0, -2.0, 1.0};
  int n = 0;
  for (int sc = 1; sc <= n_scales; ++sc) {
    const int rw = w / sc, rh = h / sc, x0 = (w - rw) / 2, y0 = (h - rh) / 2;
    for (int mi = 0; mi < per; ++mi) {
      const int m = kMembers[filter_set][mi];
      float* bw = bin_weights + (size_t)9 * n;
      for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) {
          double f = 1.0;
          if (m == HAAR2X) f = kF2[a];
          if (m == HAAR2Y) f = kF2[b];
          if (m == HAAR3X) f = kF3[a];
          if (m == HAAR3Y) f = kF3[b];
          bw[b * 3 + a] = (float)(f * g[b][a]);
        }
      vqnnf_filter_desc& d = out[n];
      d.x0 = x0;
      d.y0 = y0;
      d.x1 = x0 + rw;
      d.y1 = y0 + rh;
      d.gx = d.gy = 3;
      d.bin_weight = bw;
      d.weight = (float)((m == GAUSS ? 1.0 : 0.25) / sc);
      ++n;
    }
  }
  *n_out = n;
  return ok();
}

vqnnf_status vqnnf_template_weights(const vqnnf_template* t, float* out) {
  vqnnf_status s = check_tpl(nullptr, t);
  if (s) return s;
  if (!out) return fail(VQNNF_EINVAL, "null output");
  std::memcpy(out, t->t.weights.data(), t->t.weights.size() * sizeof(float));
  return ok();
}

vqnnf_status vqnnf_assign(vqnnf_ctx* c, const vqnnf_template* t, const vqnnf_fmap* q, int32_t prec,
                          uint8_t* labels, int64_t* n_flagged) {
  vqnnf_status s;
  if ((s = check_ctx(c)) || (s = check_tpl(c, t)) || (s = check_query(c, t, q, prec))) return s;
  prec = search_prec(prec);
  if (!labels) return fail(VQNNF_EINVAL, "null labels");
  int64_t n = (int64_t)q->H * q->W;
  if ((s = assign_scratch(c, t, n, prec, false))) return s;
  const ScaledSet* ss;
  if ((s = prepare_scaled(c, t, q, &ss))) return s;
  HookScope hs(c);
  if ((s = run_assign(c, t, q, prec, labels, false, ctx_bufs(c)))) return s;
  if (n_flagged) {
    uint32_t cnt = 0;
    if (prec == VQNNF_PREC_BF16_REFINED) {
      HIP_TRY(hipMemcpyAsync(&cnt, (char*)c->control.p + 8, 4, hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(hipStreamSynchronize(c->stream));
    }
    *n_flagged = cnt;
  }
  return ok();
}

vqnnf_status vqnnf_filter(vqnnf_ctx* c, const vqnnf_template* t, const uint8_t* labels, int32_t H,
                          int32_t W, int32_t* integral) {
  vqnnf_status s;
  if ((s = check_ctx(c)) || (s = check_tpl(c, t))) return s;
  if (!labels || !integral) return fail(VQNNF_EINVAL, "null labels or integral pointer");
  if (H < 1 || W < 1) return fail(VQNNF_EINVAL, "H and W must be >= 1");
  if ((int64_t)H * W >= (1ll << 31)) return fail(VQNNF_EINVAL, "H*W must be < 2^31");
  const int k = t->t.k;
  const int64_t R = (H + kIntTile - 1) / kIntTile, S = (W + kIntTile - 1) / kIntTile;
  size_t side = (size_t)((int64_t)H * S + R * W + R * S) * k * 4;
  if ((s = check_cap(c, {{&c->int_side, side}}))) return s;
  if ((s = need_device(c))) return s;
  if ((s = ensure(c, c->int_side, side, "integral-image side arrays"))) return s;
  IntegralArgs a{};
  a.labels = labels;
  a.H = H;
  a.W = W;
  a.k = k;
  a.P = integral;
  a.rsh = (int32_t*)c->int_side.p;
  a.cbh = a.rsh + (size_t)H * S * k;
  a.th = a.cbh + (size_t)R * W * k;
  HookScope hs(c);
  HIP_TRY(launch_integral(a, c->stream));
  return ok();
}

static vqnnf_status score_common(vqnnf_ctx* c, const vqnnf_template* t, const uint8_t* labels,
                                 const int32_t* P, int32_t H, int32_t W, float* heatmap,
                                 int32_t* best_xy, float* best_score, bool zeroed) {
  vqnnf_status s = enqueue_score(c, t, labels, P, H, W, heatmap, (unsigned long long*)c->control.p,
                                 zeroed);
  if (s) return s;
  return read_best(c, W - t->t.w + 1, best_xy, best_score);
}

vqnnf_status vqnnf_score(vqnnf_ctx* c, const vqnnf_template* t, const uint8_t* labels, int32_t H,
                         int32_t W, float* heatmap, int32_t* best_xy, float* best_score) {
  vqnnf_status s;
  if ((s = check_ctx(c)) || (s = check_tpl(c, t))) return s;
  if (!labels || !heatmap) return fail(VQNNF_EINVAL, "null labels or heatmap");
  if ((s = check_score_dims(t, H, W))) return s;
  if (!fused_supported(t->t))
    return fail(VQNNF_ENOTSUP, "on-chip scoring needs the full-window + g x g grid bank (g <= 4) "
                "with at most four distinct bin weights, within the LDS budget; use vqnnf_filter + "
                "vqnnf_score_integral");
  const size_t pb = fused_partial_bytes(t->t, H, W);
  if ((s = check_cap(c, {{&c->control, 64}, {&c->partials, pb}}))) return s;
  if ((s = need_device(c))) return s;
  if ((s = ensure(c, c->control, 64, "control block"))) return s;
  if ((s = ensure(c, c->partials, pb, "score partial sums"))) return s;
  HookScope hs(c);
  return score_common(c, t, labels, nullptr, H, W, heatmap, best_xy, best_score, false);
}

vqnnf_status vqnnf_score_integral(vqnnf_ctx* c, const vqnnf_template* t, const int32_t* integral,
                                  int32_t H, int32_t W, float* heatmap, int32_t* best_xy,
                                  float* best_score) {
  vqnnf_status s;
  if ((s = check_ctx(c)) || (s = check_tpl(c, t))) return s;
  if (!integral || !heatmap) return fail(VQNNF_EINVAL, "null integral or heatmap");
  if ((s = check_score_dims(t, H, W))) return s;
  if ((s = check_cap(c, {{&c->control, 64}}))) return s;
  if ((s = need_device(c))) return s;
  if ((s = ensure(c, c->control, 64, "control block"))) return s;
  HookScope hs(c);
  return score_common(c, t, nullptr, integral, H, W, heatmap, best_xy, best_score, false);
}

vqnnf_status vqnnf_match(vqnnf_ctx* c, const vqnnf_template* t, const vqnnf_fmap* q, int32_t prec,
                         float* heatmap, int32_t* best_xy, float* best_score) {
  vqnnf_status s;
  if ((s = check_ctx(c)) || (s = check_tpl(c, t)) || (s = check_query(c, t, q, prec))) return s;
  prec = search_prec(prec);
  if (!heatmap) return fail(VQNNF_EINVAL, "null heatmap");
  if ((s = check_score_dims(t, q->H, q->W))) return s;
  if ((s = pair_scratch(c, &t, &q, 1, prec, 64))) return s;
  const ScaledSet* ss;
  if ((s = prepare_scaled(c, t, q, &ss))) return s;
  HookScope hs(c);
  // one fill clears the best-location key and the worklist counter
  HIP_TRY(launch_fill_u32((uint32_t*)c->control.p, 0u, 4, c->stream));
  if ((s = enqueue_pair(c, t, q, prec, heatmap, (unsigned long long*)c->control.p, true))) return s;
  return read_best(c, q->W - t->t.w + 1, best_xy, best_score);
}

vqnnf_status vqnnf_match_noalloc(vqnnf_ctx* c, const vqnnf_template* t, const vqnnf_fmap* q,
                                 int32_t prec, float* heatmap, int32_t* best_xy, float* best_score) {
  vqnnf_status s;
  if ((s = check_ctx(c)) || (s = check_tpl(c, t)) || (s = check_query(c, t, q, prec))) return s;
  prec = search_prec(prec);
  if (!heatmap) return fail(VQNNF_EINVAL, "null heatmap");
  if ((s = check_score_dims(t, q->H, q->W))) return s;
  if (!fused_supported(t->t))
    return fail(VQNNF_ENOTSUP, "vqnnf_match_noalloc needs a bank the on-chip score takes (full window + "
                "g x g grid, g <= 4, at most four distinct bin weights)");
  const NoAllocLayout l = noalloc_layout(t->t, q->H, q->W, prec);
  if (l.total > kNoAllocScratchBytes)
    return fail(VQNNF_ENOMEM, "vqnnf_match_noalloc: a %dx%d map with k = %d needs %zu bytes of scratch; "
                "the fixed scratch holds %zu", q->W, q->H, t->t.k, l.total, kNoAllocScratchBytes);
  if ((s = need_device(c))) return s;
  // FP8 maps use the codebook tables of their channel scales, which only an
  // allocating call can build
  const ScaledSet* ss = nullptr;
  if (q->dtype == VQNNF_FP8_E4M3) {
    for (const ScaledSet& x : t->t.scaled)
      if (std::memcmp(x.scale.data(), q->channel_scale, sizeof(float) * t->t.D) == 0) ss = &x;
    if (!ss)
      return fail(VQNNF_EINVAL, "vqnnf_match_noalloc: the template has no tables for this FP8 map's channel "
                  "scales; one vqnnf_assign or vqnnf_match call with a map of these scales builds them");
  }
  char* base = (char*)noalloc_scratch(c->device);
  if (!base) return fail(VQNNF_EHIP, "the fixed scratch of device %d was not resolved", c->device);
  const PairBufs b{base, (uint8_t*)(base + l.labels), (uint32_t*)(base + l.wl_pix),
                   (uint32_t*)(base + l.wl_mask), base + l.partials};
  unsigned long long* key = (unsigned long long*)b.control;
  // the array keeps the previous call's contents: clear the best key and the
  // worklist counter with a kernel (graph-capturable, no memset node)
  HIP_TRY(launch_fill_u32((uint32_t*)b.control, 0u, 4, c->stream));
  if ((s = run_assign(c, t, q, prec, b.labels, true, b, false))) return s;
  if ((s = enqueue_score(c, t, b.labels, nullptr, q->H, q->W, heatmap, key, true, nullptr, b.partials, false)))
    return s;
  if (!best_xy && !best_score) return ok();
  unsigned long long hk = 0;
  HIP_TRY(hipMemcpyAsync(&hk, key, 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  const uint32_t ow = (uint32_t)(q->W - t->t.w + 1);
  const uint32_t idx = 0xFFFFFFFFu - (uint32_t)(hk & 0xFFFFFFFFu);
  if (best_xy) {
    best_xy[0] = (int32_t)(idx % ow);
    best_xy[1] = (int32_t)(idx / ow);
  }
  if (best_score) *best_score = unpack_score(hk);
  return ok();
}

}  // extern "C"

namespace {

// Pairs that share one query map (same pointer, layout and scales).
std::vector<std::vector<int>> group_by_map(int n, const vqnnf_fmap* const* q) {
  std::vector<std::vector<int>> groups;
  auto same = [](const vqnnf_fmap* a, const vqnnf_fmap* b) {
    const int64_t sa = map_stride(a);
    const int64_t sb = map_stride(b);
    return a->data == b->data && a->dtype == b->dtype && a->H == b->H && a->W == b->W &&
           a->D == b->D && sa == sb && a->channel_scale == b->channel_scale;
  };
  for (int i = 0; i < n; ++i) {
    bool placed = false;
    for (auto& gr : groups)
      if (same(q[gr[0]], q[i])) {
        gr.push_back(i);
        placed = true;
        break;
      }
    if (!placed) groups.push_back({i});
  }
  return groups;
}

int pow2_blocks(int kb) { return kb <= 1 ? 1 : kb <= 2 ? 2 : kb <= 4 ? 4 : 8; }

// Can the group's assignment run as one fused multi-template launch?
bool multi_ok(const std::vector<int>& gr, const vqnnf_template* const* t, const vqnnf_fmap* q0,
              int prec) {
  if (gr.size() < 2 || prec != VQNNF_PREC_BF16_REFINED) return false;
  if (q0->dtype != VQNNF_BF16 && q0->dtype != VQNNF_FP8_E4M3) return false;
  if (q0->D % 64 != 0) return false;
  const int eb = q0->dtype == VQNNF_BF16 ? 2 : 1, al = q0->dtype == VQNNF_BF16 ? 16 : 8;
  const int64_t st = q0->pixel_stride ? q0->pixel_stride : q0->D;
  if ((uintptr_t)q0->data % al != 0 || (st * eb) % al != 0) return false;
  int per_sb[9] = {};
  for (int i : gr) {
    if (t[i]->t.geom.kb > 8) return false;
    per_sb[pow2_blocks(t[i]->t.geom.kb)]++;
  }
  int passes = 0;   // templates of one block size share passes of 8 blocks
  for (int sb : {1, 2, 4, 8}) passes += (per_sb[sb] * sb + 7) / 8;
  return passes <= kMultiMaxPass && gr.size() <= 1024;
}

// Pass plan of one map group: templates sorted by padded block count, packed
// 8 blocks per pass; fragments, norms, pass and output tables on the device.
vqnnf_status build_multi_plan(vqnnf_ctx* c, vqnnf_ctx::MultiPlan& mp, const std::vector<int>& gr,
                              const vqnnf_template* const* t, const vqnnf_fmap* q0,
                              const std::vector<const ScaledSet*>& sets, int64_t n_pix, int64_t lab0,
                              int slot0) {
  std::vector<uint64_t> sig = {(uint64_t)q0->D, (uint64_t)q0->dtype, (uint64_t)n_pix, (uint64_t)lab0,
                               (uint64_t)slot0,
                               (uint64_t)(uintptr_t)c->m_labels.p, (uint64_t)(uintptr_t)c->m_count.p,
                               (uint64_t)(uintptr_t)c->m_wl_pix.p, (uint64_t)(uintptr_t)c->m_wl_mask.p};
  for (int i : gr) sig.insert(sig.end(), {t[i]->uid, (uint64_t)(uintptr_t)sets[i]});
  if (sig == mp.sig) return ok();
  // order: largest blocks first, stable within a size
  std::vector<int> order(gr.size());
  for (size_t k = 0; k < gr.size(); ++k) order[k] = (int)k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return pow2_blocks(t[gr[a]]->t.geom.kb) > pow2_blocks(t[gr[b]]->t.geom.kb);
  });
  std::vector<MultiPass> passes;
  std::vector<int> slot_pair;
  for (size_t k = 0; k < order.size();) {
    const int sb = pow2_blocks(t[gr[order[k]]]->t.geom.kb);
    MultiPass ps{sb, (int)slot_pair.size(), 0, 0};
    while (k < order.size() && pow2_blocks(t[gr[order[k]]]->t.geom.kb) == sb && ps.n_seg < 8 / sb) {
      slot_pair.push_back(order[k]);
      ++ps.n_seg;
      ++k;
    }
    passes.push_back(ps);
  }
  // kernels of an earlier batch may still read the plan being replaced
  HIP_TRY(hipStreamSynchronize(c->stream));
  const int ngr = t[gr[0]]->t.geom.d_pad_bf16 / 32;
  const int np = (int)passes.size();
  const size_t fbytes = (size_t)np * ngr * 2 * 8 * 64 * 16;
  vqnnf_status s;
  if ((s = ensure(c, mp.frag, fbytes, "batched codebook fragments")) ||
      (s = ensure(c, mp.cnorm, (size_t)np * 128 * 4, "batched codeword norms")) ||
      (s = ensure(c, mp.passes, (size_t)np * sizeof(MultiPass), "batched pass table")) ||
      (s = ensure(c, mp.outs, slot_pair.size() * sizeof(MultiOut), "batched output table")))
    return s;
  HIP_TRY(hipMemset(mp.frag.p, 0, fbytes));
  std::vector<float> pad((size_t)np * 128, 3.0e38f);
  HIP_TRY(hipMemcpy(mp.cnorm.p, pad.data(), pad.size() * 4, hipMemcpyHostToDevice));
  std::vector<MultiOut> outs(slot_pair.size());
  for (int pi = 0; pi < np; ++pi) {
    const MultiPass& ps = passes[pi];
    for (int sg = 0; sg < ps.n_seg; ++sg) {
      const int slot = ps.tmpl0 + sg;
      const int i = gr[slot_pair[slot]];
      const DeviceTemplate& d = t[i]->t;
      const ScaledSet* ss = sets[i];
      const int kb = d.geom.kb;
      // rows (group, term) of kb*64 fragments, placed at block sg*sb of the pass
      const uint4* src = ss ? ss->d_frag_bf16 : d.d_frag_bf16;
      uint4* dst = (uint4*)mp.frag.p + (size_t)pi * ngr * 2 * 8 * 64 + (size_t)sg * ps.sb * 64;
      HIP_TRY(hipMemcpy2D(dst, 8 * 64 * 16, src, (size_t)kb * 64 * 16, (size_t)kb * 64 * 16,
                          (size_t)ngr * 2, hipMemcpyDeviceToDevice));
      HIP_TRY(hipMemcpy((float*)mp.cnorm.p + (size_t)pi * 128 + sg * ps.sb * 16, d.d_cnorm,
                        (size_t)kb * 16 * 4, hipMemcpyDeviceToDevice));
      const BoundCoef& b = ss ? ss->bound : d.bound_bf16q;
      MultiOut& o = outs[slot];
      const int64_t px0 = lab0 + (int64_t)slot * n_pix;
      o.labels = (uint8_t*)c->m_labels.p + px0;
      o.wl_count = (uint32_t*)c->m_count.p + slot0 + slot;
      o.wl_pix = (uint32_t*)c->m_wl_pix.p + px0;
      o.wl_mask = (uint32_t*)c->m_wl_mask.p + px0 * 4;
      o.a0 = b.a0;
      o.a1 = b.a1;
      o.a2 = b.a2;
    }
  }
  HIP_TRY(hipMemcpy(mp.passes.p, passes.data(), passes.size() * sizeof(MultiPass), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(mp.outs.p, outs.data(), outs.size() * sizeof(MultiOut), hipMemcpyHostToDevice));
  mp.n_pass = np;
  mp.n_groups = ngr;
  mp.slot_pair = slot_pair;
  mp.sig = sig;
  return ok();
}

// Fused assignments of the batch: one launch per (storage, D) class covering
// every map group of that class, each map's pass plan in a device table.
struct MultiLaunch {
  bool fp8;
  int D, n_groups;
  std::vector<MultiMap> maps;
  int64_t n_tiles = 0;
  size_t tab_off = 0;                  // the map table's offset in the batch tables
};

void add_multi_map(std::vector<MultiLaunch>& ls, const vqnnf_ctx::MultiPlan& mp, const vqnnf_fmap* q0) {
  const bool fp8 = q0->dtype == VQNNF_FP8_E4M3;
  MultiLaunch* l = nullptr;
  for (MultiLaunch& x : ls)
    if (x.fp8 == fp8 && x.D == q0->D && x.n_groups == mp.n_groups) l = &x;
  if (!l) {
    ls.push_back(MultiLaunch{fp8, q0->D, mp.n_groups, {}, 0, 0});
    l = &ls.back();
  }
  MultiMap m{};
  m.q = q0->data;
  m.stride = map_stride(q0);
  m.n_pix = (int64_t)q0->H * q0->W;
  m.frag = (const uint4*)mp.frag.p;
  m.cnorm = (const float*)mp.cnorm.p;
  m.passes = (const MultiPass*)mp.passes.p;
  m.outs = (const MultiOut*)mp.outs.p;
  m.n_pass = mp.n_pass;
  m.tile0 = l->n_tiles;
  l->n_tiles += multi_tiles(m.n_pix);
  l->maps.push_back(m);
}

hipError_t enqueue_multi_launch(vqnnf_ctx* c, const MultiLaunch& l, const uint8_t* d_tab) {
  MultiArgs ma{};
  ma.kp.maps = (const MultiMap*)(d_tab + l.tab_off);
  ma.kp.n_maps = (int)l.maps.size();
  ma.kp.D = l.D;
  ma.kp.n_groups = l.n_groups;
  ma.kp.n_tiles = l.n_tiles;
  ma.fp8 = l.fp8;
  ma.variant = c->assign_variant;
  return launch_assign_multi(ma, c->stream, c->n_cu);
}

// Pair work of the fused groups after their assignment: re-score arguments,
// on-chip score items and the pairs scored one by one.
struct FusedWork {
  std::vector<AssignArgs> rescore;
  std::vector<ScoreBatchItem> score;
  std::vector<int> loose;              // pair index
  std::vector<const uint8_t*> loose_lab;
};

void fused_work(vqnnf_ctx* c, const vqnnf_ctx::MultiPlan& mp, const std::vector<int>& gr,
                const vqnnf_template* const* t, const vqnnf_fmap* const* q,
                const std::vector<const ScaledSet*>& sets, float* const* heatmaps, unsigned long long* keys,
                int64_t lab0, int slot0, FusedWork& w) {
  const vqnnf_fmap* q0 = q[gr[0]];
  const int64_t n_pix = (int64_t)q0->H * q0->W;
  for (int slot = 0; slot < (int)gr.size(); ++slot) {
    const int i = gr[mp.slot_pair[slot]];
    const DeviceTemplate& d = t[i]->t;
    const int64_t px0 = lab0 + (int64_t)slot * n_pix;
    uint8_t* lab = (uint8_t*)c->m_labels.p + px0;
    if ((size_t)i < c->batch_labels.size()) c->batch_labels[i] = {lab, n_pix};
    AssignArgs a{};
    a.q = q0->data;
    a.stride = map_stride(q0);
    a.n_pix = n_pix;
    a.D = q0->D;
    a.dtype = q0->dtype;
    a.t = &d;
    a.scale = sets[i] ? sets[i]->d_scale : nullptr;
    a.labels = lab;
    a.wl_count = (uint32_t*)c->m_count.p + slot0 + slot;
    a.wl_pix = (uint32_t*)c->m_wl_pix.p + px0;
    a.wl_mask = (uint32_t*)c->m_wl_mask.p + px0 * 4;
    a.mask_words = (pow2_blocks(d.geom.kb) + 1) / 2;   // as the fused kernel writes them
    w.rescore.push_back(a);
    if (fused_supported(d)) {
      w.score.push_back({&d, lab, q0->H, q0->W, heatmaps[i], keys + i, 0});
    } else {
      w.loose.push_back(i);
      w.loose_lab.push_back(lab);
    }
  }
}

// Window rows per tile of a batched score: the tallest tiles (least tile
// set-up per window) that still give every compute unit 8 blocks.
int batch_default_tyw(const std::vector<ScoreBatchItem>& items, int n_cu) {
  for (int cap : {256, 128, 64, 32, 16}) {
    int64_t blocks = 0;
    for (const ScoreBatchItem& it : items) {
      const int ow = it.W - it.t->w + 1, oh = it.H - it.t->h + 1;
      const int64_t nx = (ow + 255) / 256;
      blocks += nx * ((oh + std::min(cap, oh) - 1) / std::min(cap, oh)) * fused_groups(*it.t);
    }
    if (blocks >= 8LL * n_cu) return cap;
  }
  return 8;
}

std::vector<int> batch_shape_key(const std::vector<ScoreBatchItem>& items, int n_cu) {
  std::vector<int> key = {n_cu};
  for (const ScoreBatchItem& it : items) {
    const DeviceTemplate& d = *it.t;
    key.insert(key.end(), {d.w, d.h, d.grid.g, d.geom.kpad, it.H, it.W});
    for (int f = 0; f < d.n_filters; ++f) {
      uint32_t b;
      std::memcpy(&b, &d.weights[f], 4);
      key.push_back((int)b);
    }
  }
  return key;
}

// Builds the batched score tables for a tile choice (window rows per tile,
// kScoreWide for 32-channel blocks; partial sums in b_part) and appends them
// to blob at a 256-byte boundary; returns the offset.
vqnnf_status plan_batch_score(vqnnf_ctx* c, std::vector<ScoreBatchItem> items, int choice, ScoreBatchPlan& pl,
                              std::vector<uint8_t>& blob, size_t* off) {
  for (ScoreBatchItem& it : items) it.tyw = choice & (kScoreWide - 1);
  if (!plan_score_batch(items, c->b_part.p, &pl, (choice & kScoreWide) != 0))
    return fail(VQNNF_EINVAL, "batched score: a pair's bank or size is outside the on-chip kernel's range");
  *off = (blob.size() + 255) / 256 * 256;
  blob.resize(*off + pl.blob.size());
  std::memcpy(blob.data() + *off, pl.blob.data(), pl.blob.size());
  return ok();
}

}  // namespace

extern "C" {

vqnnf_status vqnnf_match_batched(vqnnf_ctx* c, int32_t n, const vqnnf_template* const* t,
                                 const vqnnf_fmap* const* q, int32_t prec, float* const* heatmaps,
                                 int32_t* best_xy, float* best_score) {
  vqnnf_status s;
  if ((s = check_ctx(c))) return s;
  if (n < 1) return fail(VQNNF_EINVAL, "n_pairs must be >= 1 (got %d)", n);
  if (!t || !q || !heatmaps) return fail(VQNNF_EINVAL, "null template, map or heatmap array");
  for (int i = 0; i < n; ++i) {
    if ((s = check_tpl(c, t[i])) || (s = check_query(c, t[i], q[i], prec)) ||
        (s = check_score_dims(t[i], q[i]->H, q[i]->W))) {
      std::string m = g_err;
      return fail(s, "pair %d: %s", i, m.c_str());
    }
    if (!heatmaps[i]) return fail(VQNNF_EINVAL, "pair %d: null heatmap", i);
  }
  prec = search_prec(prec);
  c->batch_labels.assign((size_t)n, {nullptr, 0});
  if ((s = pair_scratch(c, t, q, n, prec, 64))) return s;
  std::vector<const ScaledSet*> sets((size_t)n);
  for (int i = 0; i < n; ++i)
    if ((s = prepare_scaled(c, t[i], q[i], &sets[i]))) return s;
  if ((s = check_cap(c, {{&c->keys, (size_t)n * 8}}))) return s;
  if ((s = ensure(c, c->keys, (size_t)n * 8, "best-location keys"))) return s;
  // map groups that take the fused multi-template assignment; a group whose
  // templates need more passes than one launch holds is split
  std::vector<std::vector<int>> groups;
  for (auto& gr : group_by_map(n, q)) {
    std::vector<int> cur;
    int per_sb[9] = {};
    auto passes = [&]() {
      int p = 0;
      for (int sb : {1, 2, 4, 8}) p += (per_sb[sb] * sb + 7) / 8;
      return p;
    };
    for (int i : gr) {
      const int sb = pow2_blocks(std::min(t[i]->t.geom.kb, 8));
      per_sb[sb]++;
      if (passes() > kMultiMaxPass || cur.size() >= 1024) {
        groups.push_back(cur);
        cur.clear();
        for (int& v : per_sb) v = 0;
        per_sb[sb] = 1;
      }
      cur.push_back(i);
    }
    groups.push_back(cur);
  }
  std::vector<char> fused(groups.size(), 0);
  // the fused groups' label maps, worklists and counters one after another
  std::vector<int64_t> lab0(groups.size(), 0);
  std::vector<int> slot0(groups.size(), 0);
  size_t ml = 0;
  int nslot = 0;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    fused[gi] = multi_ok(groups[gi], t, q[groups[gi][0]], prec);
    if (!fused[gi]) continue;
    lab0[gi] = (int64_t)ml;
    slot0[gi] = nslot;
    ml += groups[gi].size() * (size_t)q[groups[gi][0]]->H * q[groups[gi][0]]->W;
    nslot += (int)groups[gi].size();
  }
  if (ml) {
    const size_t cb = std::max<size_t>(4096, (size_t)nslot * 4);
    if ((s = check_cap(c, {{&c->m_labels, ml}, {&c->m_count, cb}, {&c->m_wl_pix, ml * 4},
                           {&c->m_wl_mask, ml * 16}})) ||
        (s = ensure(c, c->m_labels, ml, "batched label maps")) ||
        (s = ensure(c, c->m_count, cb, "batched worklist counters")) ||
        (s = ensure(c, c->m_wl_pix, ml * 4, "batched re-score worklists")) ||
        (s = ensure(c, c->m_wl_mask, ml * 16, "batched candidate masks")))
      return s;
  }
  if (c->mplans.size() < groups.size()) c->mplans.resize(groups.size());
  unsigned long long* keys = (unsigned long long*)c->keys.p;
  FusedWork fw;
  std::vector<MultiLaunch> mls;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    if (!fused[gi]) continue;
    const vqnnf_fmap* q0 = q[groups[gi][0]];
    if ((s = build_multi_plan(c, c->mplans[gi], groups[gi], t, q0, sets, (int64_t)q0->H * q0->W, lab0[gi],
                              slot0[gi])))
      return s;
    fused_work(c, c->mplans[gi], groups[gi], t, q, sets, heatmaps, keys, lab0[gi], slot0[gi], fw);
    add_multi_map(mls, c->mplans[gi], q0);
  }
  // batched re-score and score tables of the fused pairs
  RescoreBatchPlan rplan;
  ScoreBatchPlan splan;
  std::vector<uint8_t> blob;
  size_t soff = 0;
  std::vector<int> bkey;
  bool tune = false;
  int tyw = 0;
  // (re)builds the tables for the cached or default tile height and uploads
  // them when they changed
  auto prepare_tables = [&]() -> vqnnf_status {
    vqnnf_status st;
    blob.clear();
    rplan = RescoreBatchPlan{};
    splan = ScoreBatchPlan{};
    if (!fw.rescore.empty()) {
      plan_rescore_batch(fw.rescore, &rplan);
      blob = rplan.blob;
    }
    for (MultiLaunch& l : mls) {
      l.tab_off = (blob.size() + 255) / 256 * 256;
      blob.resize(l.tab_off + l.maps.size() * sizeof(MultiMap));
      std::memcpy(blob.data() + l.tab_off, l.maps.data(), l.maps.size() * sizeof(MultiMap));
    }
    if (!fw.score.empty()) {
      std::vector<ScoreBatchItem> sized = fw.score;   // partial sizes do not depend on the tile height
      for (ScoreBatchItem& it : sized) it.tyw = 1;
      if (!plan_score_batch(sized, nullptr, &splan))
        return fail(VQNNF_EINVAL, "batched score: a pair's bank or size is outside the on-chip kernel's range");
      if ((st = check_cap(c, {{&c->b_part, splan.part_bytes}})) ||
          (st = ensure(c, c->b_part, std::max<size_t>(splan.part_bytes, 256), "batched score partial sums")))
        return st;
      bkey = batch_shape_key(fw.score, c->n_cu);
      auto it = c->btyw_cache.find(bkey);
      tune = it == c->btyw_cache.end() && c->autotune;
      tyw = it != c->btyw_cache.end() ? it->second : batch_default_tyw(fw.score, c->n_cu);
      if ((st = plan_batch_score(c, fw.score, tyw, splan, blob, &soff))) return st;
    }
    if (!blob.empty()) {
      if ((st = check_cap(c, {{&c->b_tab, blob.size()}})) ||
          (st = ensure(c, c->b_tab, blob.size(), "batched argument tables")))
        return st;
      if (c->b_tab_at != c->b_tab.p || c->b_tab_host != blob) {
        // kernels of an earlier batch may still read the tables being replaced
        HIP_TRY(hipStreamSynchronize(c->stream));
        HIP_TRY(hipMemcpy(c->b_tab.p, blob.data(), blob.size(), hipMemcpyHostToDevice));
        c->b_tab_host = blob;
        c->b_tab_at = c->b_tab.p;
      }
    }
    return ok();
  };
  if ((s = prepare_tables())) return s;
  // Times each candidate block width and tile height on this very call (every
  // run writes the same heatmaps and keys) and keeps the fastest for the
  // batch's shapes.
  auto tune_score = [&]() -> vqnnf_status {
    std::vector<int> cand = {tyw};
    bool any_wide = false;
    for (const ScoreBatchItem& it : fw.score) any_wide = any_wide || fused_wide_allowed(*it.t);
    for (int flag : {0, kScoreWide}) {
      if (flag && !any_wide) continue;
      for (int v : {16, 32, 64, 128, 256})
        if (std::find(cand.begin(), cand.end(), v | flag) == cand.end()) cand.push_back(v | flag);
    }
    std::vector<ScoreBatchPlan> pls(cand.size());
    std::vector<uint8_t> cblob;
    std::vector<size_t> offs(cand.size());
    vqnnf_status st;
    for (size_t ci = 0; ci < cand.size(); ++ci)
      if ((st = plan_batch_score(c, fw.score, cand[ci], pls[ci], cblob, &offs[ci]))) return st;
    // temporary tables, events and the paused timing hook are released on
    // every path out of here
    struct Scratch {
      vqnnf_ctx* c;
      Buffer tmp;
      std::vector<hipEvent_t> ev;
      ~Scratch() {
        (void)hipStreamSynchronize(c->stream);
        for (auto e : ev) (void)hipEventDestroy(e);
        if (tmp.p) {
          (void)hipFree(tmp.p);
          c->used -= tmp.bytes;
        }
        if (c->timing) {
          TimingHook h{hook_begin, hook_end, c};
          set_timing_hook(&h);
        }
      }
    } sc{c, {}, {}};
    set_timing_hook(nullptr);
    if ((st = ensure(c, sc.tmp, cblob.size(), "autotuning argument tables"))) return st;
    HIP_TRY(hipMemcpyAsync(sc.tmp.p, cblob.data(), cblob.size(), hipMemcpyHostToDevice, c->stream));
    for (size_t i = 0; i < 2 * cand.size(); ++i) {
      hipEvent_t e = nullptr;
      HIP_TRY(hipEventCreate(&e));
      sc.ev.push_back(e);
    }
    const std::vector<hipEvent_t>& ev = sc.ev;
    for (int rep = 0; rep < 2; ++rep)
      for (size_t ci = 0; ci < cand.size(); ++ci) {
        if (rep == 1) HIP_TRY(hipEventRecord(ev[2 * ci], c->stream));
        HIP_TRY(launch_score_batch(pls[ci], (const uint8_t*)sc.tmp.p + offs[ci], c->stream));
        if (rep == 1) HIP_TRY(hipEventRecord(ev[2 * ci + 1], c->stream));
      }
    HIP_TRY(hipEventSynchronize(ev.back()));
    float best_ms = 1e30f;
    int best = tyw;
    for (size_t ci = 0; ci < cand.size(); ++ci) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, ev[2 * ci], ev[2 * ci + 1]));
      if (ms < best_ms) {
        best_ms = ms;
        best = cand[ci];
      }
    }
    c->btyw_cache[bkey] = best;
    return save_tune_file(c);   // the last candidate's run already produced the result
  };
  auto enqueue_all = [&]() -> vqnnf_status {
    HIP_TRY(launch_fill_u32((uint32_t*)keys, 0u, 2 * (int64_t)n, c->stream));
    if (nslot) HIP_TRY(launch_fill_u32((uint32_t*)c->m_count.p, 0u, nslot, c->stream));
    const uint8_t* d_tab = (const uint8_t*)c->b_tab.p;
    for (const MultiLaunch& l : mls) HIP_TRY(enqueue_multi_launch(c, l, d_tab));
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      if (fused[gi]) continue;
      for (int i : groups[gi]) {
        vqnnf_status st = enqueue_pair(c, t[i], q[i], prec, heatmaps[i], keys + i, false);
        if (st) return st;
      }
    }
    if (!rplan.launches.empty()) HIP_TRY(launch_rescore_batch(rplan, d_tab, c->n_cu, c->stream));
    if (!splan.launches.empty()) {
      if (tune && !c->capturing) {
        tune = false;
        vqnnf_status st = tune_score();
        if (st) return st;
      } else {
        HIP_TRY(launch_score_batch(splan, d_tab + soff, c->stream));
      }
    }
    for (size_t li = 0; li < fw.loose.size(); ++li) {
      const int i = fw.loose[li];
      vqnnf_status st = enqueue_score_labels(c, t[i], fw.loose_lab[li], q[i]->H, q[i]->W, heatmaps[i], keys + i);
      if (st) return st;
    }
    return ok();
  };
  if (!c->graph) {
    HookScope hs(c);
    if ((s = enqueue_all())) return s;
  } else {
    // shapes not tuned yet are tuned by one eager run before the capture
    bool untuned = tune;
    for (size_t gi = 0; gi < groups.size() && c->autotune; ++gi) {
      if (fused[gi]) continue;   // pairs scored one by one
      for (int i : groups[gi]) {
        const DeviceTemplate& d = t[i]->t;
        if (!fused_supported(d)) continue;
        bool uni = true;
        for (int f = 2; f < d.n_filters; ++f) uni = uni && d.weights[f] == d.weights[1];
        const std::vector<int> key = {d.w, d.h, d.grid.g, d.geom.kpad, q[i]->H, q[i]->W, uni ? 1 : 0};
        untuned = untuned || c->tyw_cache.find(key) == c->tyw_cache.end();
      }
    }
    if (untuned) {
      HookScope hs(c);
      if ((s = enqueue_all())) return s;
      if ((s = prepare_tables())) return s;
    }
    // every argument the captured kernels depend on, scratch and plans included
    std::vector<uint64_t> sig = {(uint64_t)n, (uint64_t)prec, (uint64_t)(uintptr_t)c->stream,
                                 (uint64_t)(uintptr_t)c->control.p, (uint64_t)(uintptr_t)c->labels.p,
                                 (uint64_t)(uintptr_t)c->wl_pix.p, (uint64_t)(uintptr_t)c->wl_mask.p,
                                 (uint64_t)(uintptr_t)c->partials.p, (uint64_t)(uintptr_t)c->int_side.p,
                                 (uint64_t)(uintptr_t)c->int_p.p, (uint64_t)(uintptr_t)keys,
                                 (uint64_t)(uintptr_t)c->m_labels.p, (uint64_t)(uintptr_t)c->m_count.p,
                                 (uint64_t)(uintptr_t)c->m_wl_pix.p, (uint64_t)(uintptr_t)c->m_wl_mask.p};
    sig.insert(sig.end(), {(uint64_t)(uintptr_t)c->b_part.p, (uint64_t)(uintptr_t)c->b_tab.p,
                           (uint64_t)blob.size(), (uint64_t)soff, (uint64_t)tyw});
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      sig.push_back(fused[gi] ? 1u : 0u);
      if (fused[gi]) {
        const auto& mp = c->mplans[gi];
        sig.insert(sig.end(), {(uint64_t)(uintptr_t)mp.frag.p, (uint64_t)(uintptr_t)mp.cnorm.p,
                               (uint64_t)(uintptr_t)mp.passes.p, (uint64_t)(uintptr_t)mp.outs.p});
        sig.insert(sig.end(), mp.sig.begin(), mp.sig.end());
      }
    }
    for (int i = 0; i < n; ++i) {
      const vqnnf_fmap& m = *q[i];
      sig.insert(sig.end(), {t[i]->uid, (uint64_t)(uintptr_t)m.data, (uint64_t)m.dtype,
                             (uint64_t)m.H, (uint64_t)m.W, (uint64_t)m.D, (uint64_t)m.pixel_stride,
                             (uint64_t)(uintptr_t)sets[i], (uint64_t)(uintptr_t)heatmaps[i]});
    }
    if (!(c->gexec && sig == c->gsig)) {
      if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
      // the capture stream waits for earlier work on the context stream
      HIP_TRY(hipStreamSynchronize(c->stream));
      HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
      hipStream_t user = c->stream;
      c->stream = c->cap_stream;
      c->capturing = true;
      vqnnf_status st = enqueue_all();
      c->capturing = false;
      c->stream = user;
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
      if (st) {
        if (g) hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess) return fail(VQNNF_EHIP, "graph capture: %s", hipGetErrorString(e));
      hipGraphExec_t ex = nullptr;
      e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if (e != hipSuccess) return fail(VQNNF_EHIP, "graph instantiate: %s", hipGetErrorString(e));
      if (c->gexec) hipGraphExecDestroy(c->gexec);
      c->gexec = ex;
      c->gsig = sig;
    }
    HIP_TRY(hipGraphLaunch(c->gexec, c->stream));
  }
  if (!best_xy && !best_score) return ok();
  std::vector<unsigned long long> hk((size_t)n);
  HIP_TRY(hipMemcpyAsync(hk.data(), keys, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int i = 0; i < n; ++i) {
    const uint32_t ow = (uint32_t)(q[i]->W - t[i]->t.w + 1);
    const uint32_t idx = 0xFFFFFFFFu - (uint32_t)(hk[i] & 0xFFFFFFFFu);
    if (best_xy) {
      best_xy[2 * i] = (int32_t)(idx % ow);
      best_xy[2 * i + 1] = (int32_t)(idx / ow);
    }
    if (best_score) best_score[i] = unpack_score(hk[i]);
  }
  return ok();
}

vqnnf_status vqnnf_ctx_set_tune_file(vqnnf_ctx* c, const char* path) {
  vqnnf_status s;
  if ((s = check_ctx(c))) return s;
  c->tune_file = path ? path : "";
  if (!path) return ok();
  // lines "<kind> <compute units> <key ints ...> <value>"; kinds a (assignment
  // schedule), s (tile height of a single score), b (of a batched score);
  // entries of other compute-unit counts and malformed lines are skipped
  FILE* f = std::fopen(path, "r");
  if (!f) return ok();   // nothing tuned yet
  char line[4096];
  while (std::fgets(line, sizeof(line), f)) {
    char kind = 0;
    int off = 0;
    if (std::sscanf(line, " %c%n", &kind, &off) != 1 || (kind != 'a' && kind != 's' && kind != 'b')) continue;
    std::vector<long long> v;
    const char* p = line + off;
    for (;;) {
      long long x;
      int n = 0;
      if (std::sscanf(p, " %lld%n", &x, &n) != 1) break;
      v.push_back(x);
      p += n;
    }
    if (v.size() < 3 || v[0] != c->n_cu) continue;
    std::vector<int> key(v.begin() + 1, v.end() - 1);
    const int val = (int)v.back();
    if (val < 1) continue;
    if (kind == 'a') c->avar_cache[key] = val;
    else if (kind == 's') c->tyw_cache[key] = val;
    else c->btyw_cache[key] = val;
  }
  std::fclose(f);
  return ok();
}

vqnnf_status vqnnf_batched_labels(vqnnf_ctx* c, int32_t pair, uint8_t* labels) {
  vqnnf_status s;
  if ((s = check_ctx(c))) return s;
  if (!labels) return fail(VQNNF_EINVAL, "null labels");
  if (pair < 0 || (size_t)pair >= c->batch_labels.size())
    return fail(VQNNF_EINVAL, "pair %d is outside the last batched call (%zu pairs)", pair, c->batch_labels.size());
  const auto& e = c->batch_labels[pair];
  if (!e.first)
    return fail(VQNNF_ENOTSUP, "pair %d was matched on its own; its label map is not kept", pair);
  if ((s = need_device(c))) return s;
  HIP_TRY(hipMemcpyAsync(labels, e.first, (size_t)e.second, hipMemcpyDeviceToDevice, c->stream));
  return ok();
}

vqnnf_status vqnnf_ctx_set_debug_scores(vqnnf_ctx* c, float* scores, int64_t capacity) {
  vqnnf_status s;
  if ((s = check_ctx(c))) return s;
  if (scores && capacity < 1) return fail(VQNNF_EINVAL, "capacity must be >= 1");
  c->dbg_scores = scores;
  c->dbg_cap = scores ? capacity : 0;
  return ok();
}

vqnnf_status vqnnf_template_score_bound(const vqnnf_template* t, int32_t dtype, const float* channel_scale,
                                        double* out) {
  vqnnf_status s = check_tpl(nullptr, t);
  if (s) return s;
  if (!out) return fail(VQNNF_EINVAL, "null output");
  BoundCoef b;
  if (dtype == VQNNF_BF16) {
    b = t->t.bound_bf16q;
  } else if (dtype == VQNNF_F32) {
    b = t->t.bound_f32q;
  } else if (dtype == VQNNF_FP8_E4M3) {
    if (!channel_scale) return fail(VQNNF_EINVAL, "FP8 needs channel_scale");
    for (int d = 0; d < t->t.D; ++d)
      if (!std::isfinite(channel_scale[d]) || channel_scale[d] < 0.0f)
        return fail(VQNNF_EINVAL, "channel_scale[%d] must be finite and >= 0", d);
    std::vector<uint16_t> fb;
    std::vector<float> ff;
    build_scaled_tables(t->t, channel_scale, fb, ff, b);
  } else {
    return fail(VQNNF_EINVAL, "dtype %d has no matrix-core bound", dtype);
  }
  out[0] = b.a0;
  out[1] = b.a1;
  out[2] = b.a2;
  out[3] = b.A0;
  out[4] = b.A1;
  return ok();
}

vqnnf_status vqnnf_ctx_set_autotune(vqnnf_ctx* c, int32_t enable) {
  vqnnf_status s = check_ctx(c);
  if (s) return s;
  c->autotune = enable != 0;
  if (!c->autotune) {
    c->tyw_cache.clear();
    c->btyw_cache.clear();
    c->avar_cache.clear();
  }
  return ok();
}

vqnnf_status vqnnf_ctx_set_graph(vqnnf_ctx* c, int32_t enable) {
  vqnnf_status s = check_ctx(c);
  if (s) return s;
  if ((s = need_device(c))) return s;
  c->graph = enable != 0;
  if (!c->graph && c->gexec) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    c->gsig.clear();
  }
  return ok();
}

vqnnf_status vqnnf_ctx_set_timing(vqnnf_ctx* c, int32_t enable) {
  vqnnf_status s = check_ctx(c);
  if (s) return s;
  if ((s = need_device(c))) return s;
  if (!enable && c->timing) collect_times(c);
  c->timing = enable != 0;
  return ok();
}

vqnnf_status vqnnf_ctx_kernel_times(vqnnf_ctx* c, int32_t max_entries, const char** names,
                                    int64_t* launches, double* total_ms, int32_t* n_entries) {
  vqnnf_status s = check_ctx(c);
  if (s) return s;
  if ((s = need_device(c))) return s;
  if ((s = collect_times(c))) return s;
  int n = 0;
  for (int i = 0; i < K_COUNT; ++i) {
    if (c->launches[i] == 0) continue;
    if (n < max_entries) {
      if (names) names[n] = kernel_name(i);
      if (launches) launches[n] = c->launches[i];
      if (total_ms) total_ms[n] = c->total_ms[i];
    }
    ++n;
  }
  if (n_entries) *n_entries = n;
  return ok();
}

vqnnf_status vqnnf_ctx_reset_times(vqnnf_ctx* c) {
  vqnnf_status s = check_ctx(c);
  if (s) return s;
  if ((s = need_device(c))) return s;
  if ((s = collect_times(c))) return s;
  for (int i = 0; i < K_COUNT; ++i) {
    c->launches[i] = 0;
    c->total_ms[i] = 0;
  }
  return ok();
}

}  // extern "C"
