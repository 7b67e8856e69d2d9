// Host-side exercise of the library under AddressSanitizer and
// UndefinedBehaviorSanitizer (built by tests/test_host_sanitizers.py): a
// device-less context, template preparation on the host (k-means, NNF,
// counts, weighted banks, RGB templates), every getter, PCA, and the
// argument checks of the GPU calls, none of which reaches the device.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "vqnnf.h"

static int fails = 0;
#define EXPECT(cond)                                                           \
  do {                                                                         \
    if (!(cond)) {                                                             \
      std::fprintf(stderr, "line %d: %s (%s)\n", __LINE__, #cond, vqnnf_last_error()); \
      ++fails;                                                                 \
    }                                                                          \
  } while (0)

static float lcg(uint32_t& s) {
  s = s * 1664525u + 1013904223u;
  return (float)((s >> 8) & 0xFFFF) / 65536.0f - 0.5f;
}

int main() {
  vqnnf_ctx* ctx = nullptr;
  EXPECT(vqnnf_ctx_create_host(0, &ctx) == VQNNF_OK && ctx);
  uint32_t seed = 12345u;
  const int h = 12, w = 10, D = 20, k = 6;
  std::vector<float> tmpl((size_t)h * w * D);
  for (float& v : tmpl) v = lcg(seed);
  vqnnf_fmap tm{tmpl.data(), VQNNF_F32, h, w, D, 0, nullptr};
  vqnnf_filter_desc bank[2] = {{0, 0, w, h, 1, 1, nullptr, 1.0f}, {0, 0, w, h, 3, 3, nullptr, 1.0f}};
  vqnnf_template* t = nullptr;
  EXPECT(vqnnf_codebook(ctx, &tm, k, 20, 7, bank, 2, &t) == VQNNF_OK && t);
  int32_t tw, th, tD, tk, nf;
  EXPECT(vqnnf_template_info(t, &tw, &th, &tD, &tk, &nf) == VQNNF_OK && nf == 10);
  std::vector<float> cb((size_t)k * D), wts(nf), resp((size_t)nf * k);
  std::vector<uint8_t> lab((size_t)h * w);
  std::vector<int32_t> cnt((size_t)nf * k);
  EXPECT(vqnnf_template_codebook(t, cb.data()) == VQNNF_OK);
  EXPECT(vqnnf_template_labels(t, lab.data()) == VQNNF_OK);
  EXPECT(vqnnf_template_counts(t, cnt.data()) == VQNNF_OK);
  EXPECT(vqnnf_template_weights(t, wts.data()) == VQNNF_OK);
  EXPECT(vqnnf_template_responses(t, resp.data()) == VQNNF_OK);
  int64_t total = 0;
  for (int j = 0; j < k; ++j) total += cnt[j];
  EXPECT(total == (int64_t)h * w);
  double bound[5];
  EXPECT(vqnnf_template_score_bound(t, VQNNF_BF16, nullptr, bound) == VQNNF_OK && bound[0] > 0.0);
  std::vector<float> scale(D, 0.01f);
  EXPECT(vqnnf_template_score_bound(t, VQNNF_FP8_E4M3, scale.data(), bound) == VQNNF_OK);
  // the same codebook restored, a weighted bank (the paper's filters)
  vqnnf_filter_desc pb[10];
  float bw[90];
  int32_t n_out = 0;
  EXPECT(vqnnf_paper_bank(w, h, VQNNF_BANK_23RECT, 2, pb, bw, 10, &n_out) == VQNNF_OK && n_out == 10);
  vqnnf_template* t2 = nullptr;
  EXPECT(vqnnf_template_from_codebook(ctx, &tm, cb.data(), k, pb, n_out, &t2) == VQNNF_OK);
  std::vector<float> resp2((size_t)10 * k);
  EXPECT(vqnnf_template_responses(t2, resp2.data()) == VQNNF_OK);
  EXPECT(vqnnf_template_counts(t2, cnt.data()) == VQNNF_ENOTSUP);
  // an RGB template (colour features built on the host)
  std::vector<uint8_t> rgb((size_t)h * w * 3);
  for (uint8_t& v : rgb) v = (uint8_t)(seed = seed * 1103515245u + 12345u) >> 3;
  vqnnf_fmap rm{rgb.data(), VQNNF_RGB8, h, w, 27, 0, nullptr};
  vqnnf_template* t3 = nullptr;
  EXPECT(vqnnf_codebook(ctx, &rm, 5, 5, 3, bank, 2, &t3) == VQNNF_OK);
  // PCA
  std::vector<float> mean(D), basis((size_t)4 * D), var(4);
  EXPECT(vqnnf_pca_fit(&tm, 4, mean.data(), basis.data(), var.data()) == VQNNF_OK);
  EXPECT(var[0] >= var[1] && var[1] >= var[2]);
  // batched template preparation on the host
  const vqnnf_fmap* maps[2] = {&tm, &tm};
  const int32_t ks[2] = {3, 4};
  const uint64_t seeds[2] = {1, 2};
  const vqnnf_filter_desc* banks[2] = {bank, bank};
  const int32_t nds[2] = {2, 2};
  vqnnf_template* tb[2] = {nullptr, nullptr};
  EXPECT(vqnnf_codebook_batched(ctx, 2, maps, ks, 10, seeds, banks, nds, tb) == VQNNF_OK);
  // argument checks of the GPU calls: every one fails before any device work
  uint8_t* dummy = (uint8_t*)0x1000;
  vqnnf_fmap q{dummy, VQNNF_BF16, 64, 64, D, 0, nullptr};
  float* heat = (float*)0x2000;
  int32_t bxy[2];
  float bs;
  EXPECT(vqnnf_match(ctx, t, &q, VQNNF_PREC_BF16_REFINED, heat, bxy, &bs) == VQNNF_ENOTSUP);
  EXPECT(vqnnf_match_noalloc(ctx, t, &q, VQNNF_PREC_BF16_REFINED, heat, bxy, &bs) == VQNNF_ENOTSUP);
  q.D = D + 1;
  EXPECT(vqnnf_match(ctx, t, &q, VQNNF_PREC_BF16_REFINED, heat, bxy, &bs) == VQNNF_EINVAL);
  q.D = D;
  q.H = 5;
  EXPECT(vqnnf_match(ctx, t, &q, VQNNF_PREC_BF16_REFINED, heat, bxy, &bs) == VQNNF_EINVAL);
  q.H = 64;
  EXPECT(vqnnf_match(ctx, t, &q, 7, heat, bxy, &bs) == VQNNF_EINVAL);
  EXPECT(vqnnf_assign(ctx, t, &q, VQNNF_PREC_FP8_REFINED, dummy, nullptr) == VQNNF_EINVAL);
  EXPECT(vqnnf_assign(ctx, t, &q, VQNNF_PREC_BF16_REFINED, nullptr, nullptr) == VQNNF_EINVAL);
  EXPECT(vqnnf_filter(ctx, t, nullptr, 8, 8, nullptr) == VQNNF_EINVAL);
  const vqnnf_template* tt[1] = {t};
  const vqnnf_fmap* qq[1] = {&q};
  float* hh[1] = {heat};
  EXPECT(vqnnf_match_batched(ctx, 1, tt, qq, VQNNF_PREC_BF16_REFINED, hh, bxy, &bs) == VQNNF_ENOTSUP);
  EXPECT(vqnnf_batched_labels(ctx, 5, dummy) == VQNNF_EINVAL);
  vqnnf_template* bad = t;
  EXPECT(vqnnf_codebook(ctx, &tm, 0, 20, 1, bank, 2, &bad) == VQNNF_EINVAL && bad == nullptr);
  // handles: freed exactly once; use after free is reported
  vqnnf_template_free(t);
  vqnnf_template_free(t2);
  vqnnf_template_free(t3);
  vqnnf_template_free(tb[0]);
  vqnnf_template_free(tb[1]);
  vqnnf_ctx_destroy(ctx);
  if (fails) {
    std::fprintf(stderr, "%d checks failed\n", fails);
    return 1;
  }
  std::printf("host sanitizer driver: all checks passed\n");
  return 0;
}
