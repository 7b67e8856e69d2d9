"""Batched matching (vqnnf_match_batched) through the C ABI.

The batch runs the same kernels as single-pair matching, so every heatmap
and best location must equal what vqnnf_match gives for that pair, bit for
bit; two pairs of each batch are also checked against the FP64 oracle
(labels exact, heatmap within the parity tolerance).  Graph mode must
reproduce the eager results on every replay, with other work on the stream
in between, and re-capture when the arguments change."""
import sys

import numpy as np
import pytest

from oracle import vqnnf_oracle as O
from paper_2306_15010_amd import binding as B
from paper_2306_15010_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL, ABS = 1e-5, 4 * 2.0 ** -24


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    c = B.Context(stream=torch.cuda.current_stream())
    yield c
    torch.cuda.synchronize()
    c.close()


def to_dev(qm):
    if qm.dtype == "f32":
        return torch.from_numpy(np.ascontiguousarray(qm.data)).cuda()
    return torch.from_numpy(qm.data.view(np.int16)).cuda()


def make_pairs(ctx, wl, odd_bank_at=None):
    """Template handles, device maps and heatmap buffers for every (map, template)."""
    tpls, fms, heats, meta = [], [], [], []
    devs = [to_dev(qm) for qm in wl.maps]
    for mi, (qm, row) in enumerate(zip(wl.maps, wl.templates)):
        for ti, t in enumerate(row):
            h, w, _ = t.data.shape
            if odd_bank_at == (mi, ti):
                # a bank the on-chip kernel does not take: integral-image path
                bank = [(0, 0, w, h, 1, 1, 1.0), (0, 0, w // 2 + 1, h, 1, 2, 0.5)]
            else:
                bank = B.default_bank(w, h, t.grid)
            tpls.append(B.vqnnf_codebook(ctx, t.data, t.k, 20, 0, bank))
            fms.append(B.device_fmap(devs[mi], qm.dtype))
            heats.append(torch.full(((qm.H - h + 1) * (qm.W - w + 1),), float("nan"), device="cuda"))
            meta.append((mi, ti, bank))
    return tpls, fms, heats, meta, devs


def per_pair(ctx, tpls, fms, heats, prec):
    refs, bests = [], []
    for tp, fm, ht in zip(tpls, fms, heats):
        r = torch.empty_like(ht)
        bests.append(B.vqnnf_match(ctx, tp, fm, prec, r))
        refs.append(r)
    return refs, bests


def check_oracle(wl, tp, mi, ti, bank, heat):
    qm, t = wl.maps[mi], wl.templates[mi][ti]
    h, w, _ = t.data.shape
    # the oracle's own k-means (make_pairs asks for 20 iterations, seed 0)
    cb32 = O.kmeans_codebook(t.data, t.k, 20, 0)
    assert np.array_equal(tp.codebook().view(np.uint32), cb32.view(np.uint32))
    cb = cb32.astype(np.float64)
    labels = O.assign_map(O.decode(qm.dtype, qm.data, qm.scale), cb)
    filters = O.expand_bank([O.FilterDesc(*b[:6], None, b[6]) for b in bank])
    rt = O.template_representation(O.assign_map(t.data.astype(np.float64), cb), t.k, filters)
    sim = O.similarity_map_fast(labels, t.k, w, h, filters, rt)
    gpu = heat.cpu().numpy().reshape(sim.shape).astype(np.float64)
    err = np.abs(gpu - sim)
    log(f"pair (map {mi}, template {ti}) vs oracle: max abs err {err.max():.3e}")
    assert (err <= REL * np.abs(sim) + ABS).all()


@pytest.mark.parametrize("prec", [B.VQNNF_PREC_BF16_REFINED, B.VQNNF_PREC_FP32_PLAIN])
def test_batched_one_map_many_templates(ctx, prec):
    wl = synth.make_multi_template(41, 160, 192, 64, 32, 0.3, "bf16", 6, (12, 48), (16, 32, 64), 2)
    tpls, fms, heats, meta, _ = make_pairs(ctx, wl, odd_bank_at=(0, 3))
    log("batched: 6 templates on one 160x192 map, prec", prec)
    out = B.vqnnf_match_batched(ctx, tpls, fms, prec, heats)
    refs, bests = per_pair(ctx, tpls, fms, heats, prec)
    for i in range(len(tpls)):
        assert torch.equal(heats[i], refs[i]), f"pair {i}"
        assert out[i] == bests[i], f"pair {i}: {out[i]} vs {bests[i]}"
    if prec == B.VQNNF_PREC_BF16_REFINED:
        for i in (0, 3):
            check_oracle(wl, tpls[i], *meta[i], heats[i])


def test_batched_fused_pass_packing(ctx):
    """13 templates on one map: k = 48 pads to 4 blocks, k = 128 fills a pass,
    k = 16 templates spill into a second pass of their size."""
    wl = synth.make_multi_template(53, 96, 112, 128, 32, 0.3, "bf16", 13, (10, 32), (16, 48, 128, 32), 2)
    ks = sorted(t.k for t in wl.templates[0])
    log("k per template:", ks)
    tpls, fms, heats, meta, _ = make_pairs(ctx, wl)
    P = B.VQNNF_PREC_BF16_REFINED
    out = B.vqnnf_match_batched(ctx, tpls, fms, P, heats)
    refs, bests = per_pair(ctx, tpls, fms, heats, P)
    for i in range(len(tpls)):
        assert torch.equal(heats[i], refs[i]), f"pair {i} (k={tpls[i].k})"
        assert out[i] == bests[i]
    for i in (ks.index(128) if 128 in ks else 0, len(tpls) - 1):
        check_oracle(wl, tpls[i], *meta[i], heats[i])


def test_batched_uneven_maps(ctx):
    wl = synth.make_multi_map(43, 3, (64, 192), 48, 32, 0.3, "bf16", 2, (16, 40), 32, 3)
    tpls, fms, heats, meta, _ = make_pairs(ctx, wl)
    log("batched: maps", [(m.H, m.W) for m in wl.maps])
    out = B.vqnnf_match_batched(ctx, tpls, fms, B.VQNNF_PREC_BF16_REFINED, heats)
    refs, bests = per_pair(ctx, tpls, fms, heats, B.VQNNF_PREC_BF16_REFINED)
    for i in range(len(tpls)):
        assert torch.equal(heats[i], refs[i]), f"pair {i}"
        assert out[i] == bests[i]
    for i in (1, len(tpls) - 1):
        check_oracle(wl, tpls[i], *meta[i], heats[i])
    # the planted crops are found
    for i, (mi, ti, _) in enumerate(meta):
        t = wl.templates[mi][ti]
        assert out[i][0] == (t.x0, t.y0), (i, out[i], (t.x0, t.y0))


def test_batched_graph_replays(ctx):
    wl = synth.make_multi_template(47, 128, 144, 64, 32, 0.3, "bf16", 4, (12, 40), (16, 32), 2)
    tpls, fms, heats, meta, devs = make_pairs(ctx, wl)
    P = B.VQNNF_PREC_BF16_REFINED
    eager = B.vqnnf_match_batched(ctx, tpls, fms, P, heats)
    ref = [h.clone() for h in heats]
    B.vqnnf_ctx_set_graph(ctx, True)
    try:
        for rep in range(3):
            for h in heats:
                h.fill_(float("nan"))
            log("graph replay", rep)
            out = B.vqnnf_match_batched(ctx, tpls, fms, P, heats)
            torch.cuda.synchronize()
            assert out == eager
            for i in range(len(heats)):
                assert torch.equal(heats[i], ref[i]), (rep, i)
            # eager work on the same stream between replays
            tmp = torch.empty_like(heats[0])
            B.vqnnf_match(ctx, tpls[0], fms[0], P, tmp)
            torch.cuda.synchronize()
        # new output buffers: a new signature, captured again
        heats2 = [torch.full_like(h, float("nan")) for h in heats]
        out = B.vqnnf_match_batched(ctx, tpls, fms, P, heats2)
        assert out == eager
        for i in range(len(heats)):
            assert torch.equal(heats2[i], ref[i])
        # input contents change, arguments do not: the replay sees the new data
        devs[0].copy_(torch.flip(devs[0], dims=[0]))
        out_flip = B.vqnnf_match_batched(ctx, tpls, fms, P, heats2)
    finally:
        B.vqnnf_ctx_set_graph(ctx, False)
    refs, bests = per_pair(ctx, tpls, fms, heats2, P)
    assert out_flip == bests
    for i in range(len(heats)):
        assert torch.equal(heats2[i], refs[i])


def test_autotune_keeps_results(ctx):
    """The tile height changes only the schedule: the default, the tuning call
    and the cached choice give the same heatmap bit for bit, and so does a
    graph captured right after its tuning run."""
    wl = synth.make_multi_template(59, 200, 176, 64, 32, 0.3, "bf16", 2, (20, 40), (32, 64), 3)
    tpls, fms, heats, meta, _ = make_pairs(ctx, wl)
    P = B.VQNNF_PREC_BF16_REFINED
    B.vqnnf_ctx_set_autotune(ctx, False)
    ref = B.vqnnf_match_batched(ctx, tpls, fms, P, heats)
    ref_h = [h.clone() for h in heats]
    B.vqnnf_ctx_set_graph(ctx, True)
    try:
        B.vqnnf_ctx_set_autotune(ctx, True)     # empty cache: an eager run tunes, then capture
        assert B.vqnnf_match_batched(ctx, tpls, fms, P, heats) == ref
        assert all(torch.equal(a, b) for a, b in zip(heats, ref_h))
    finally:
        B.vqnnf_ctx_set_graph(ctx, False)
    for rep in range(2):                        # first: tunes on this call, then cached
        for h in heats:
            h.fill_(float("nan"))
        assert B.vqnnf_match_batched(ctx, tpls, fms, P, heats) == ref, rep
        assert all(torch.equal(a, b) for a, b in zip(heats, ref_h)), rep


def test_batched_mask_words_and_classes(ctx):
    """Codebook sizes whose padded block count is not a power of two (k = 80,
    96: the fused kernel writes four candidate-mask words per pixel) next to
    k = 8 (one channel group: the tile kernel forms the score itself), with
    3 x 3 grids over sides not divisible by 3 (bins of unequal area: sums
    merged by weight)."""
    wl = synth.make_multi_template(61, 120, 136, 64, 24, 0.3, "bf16", 7, (19, 44), (80, 96, 8, 48), 3)
    tpls, fms, heats, meta, _ = make_pairs(ctx, wl)
    log("k per template:", [t.k for t in wl.templates[0]], "sides:", [t.data.shape[0] for t in wl.templates[0]])
    P = B.VQNNF_PREC_BF16_REFINED
    out = B.vqnnf_match_batched(ctx, tpls, fms, P, heats)
    refs, bests = per_pair(ctx, tpls, fms, heats, P)
    for i in range(len(tpls)):
        assert torch.equal(heats[i], refs[i]), f"pair {i} (k={tpls[i].k})"
        assert out[i] == bests[i]
    for i in range(len(tpls)):
        check_oracle(wl, tpls[i], *meta[i], heats[i])


def test_largest_template(ctx):
    """Templates of the largest side (255): the per-group sums of a window
    reach their 16-bit storage's largest values (single and batched)."""
    wl = synth.make_multi_template(67, 290, 300, 16, 12, 0.3, "bf16", 2, (255, 255), (32, 48), 2)
    tpls, fms, heats, meta, _ = make_pairs(ctx, wl)
    log("sides:", [t.data.shape[:2] for t in wl.templates[0]])
    P = B.VQNNF_PREC_BF16_REFINED
    out = B.vqnnf_match_batched(ctx, tpls, fms, P, heats)
    refs, bests = per_pair(ctx, tpls, fms, heats, P)
    for i in range(len(tpls)):
        assert torch.equal(heats[i], refs[i]), f"pair {i}"
        assert out[i] == bests[i]
        check_oracle(wl, tpls[i], *meta[i], heats[i])


def test_batched_many_maps_one_launch(ctx):
    """Maps of uneven size (one smaller than a tile row of the chip) and two
    feature sizes: one fused assignment launch per feature size, each block
    walking a contiguous run of tiles that crosses map boundaries."""
    wa = synth.make_multi_map(71, 4, (24, 200), 64, 24, 0.3, "bf16", 3, (8, 20), 16, 2)
    wb = synth.make_multi_map(73, 3, (40, 160), 128, 24, 0.3, "bf16", 2, (10, 24), 32, 3)
    pa = make_pairs(ctx, wa)
    pb = make_pairs(ctx, wb)
    tpls, fms, heats = pa[0] + pb[0], pa[1] + pb[1], pa[2] + pb[2]
    log("maps:", [(m.H, m.W, m.D) for m in wa.maps + wb.maps])
    P = B.VQNNF_PREC_BF16_REFINED
    out = B.vqnnf_match_batched(ctx, tpls, fms, P, heats)
    refs, bests = per_pair(ctx, tpls, fms, heats, P)
    for i in range(len(tpls)):
        assert torch.equal(heats[i], refs[i]), f"pair {i}"
        assert out[i] == bests[i]
    check_oracle(wa, tpls[0], *pa[3][0], heats[0])
    n_a = len(pa[0])
    check_oracle(wb, tpls[n_a + 1], *pb[3][1], heats[n_a + 1])


def test_batched_mixed_storage(ctx):
    """One batch over an FP32 map (D = 64), a low-dimensional FP32 map
    (D = 18), a BF16 map (D = 128) and an RGB image (colour features,
    D = 27): maps that share the fused assignment launch and maps that take
    their own assignment kernels.  Every pair equals its single-pair
    vqnnf_match bit for bit; the FP32, low-D and RGB pairs are checked
    against the oracle (its own k-means and colour features)."""
    P = B.VQNNF_PREC_BF16_REFINED
    rng = np.random.default_rng(75)
    pairs = []   # (template handle, fmap, heatmap, oracle query features, oracle template features, k, w, h, seed)
    devs = []

    def add_float_map(qm, sides, k):
        q64 = O.decode(qm.dtype, qm.data, qm.scale)
        dev = to_dev(qm)
        devs.append(dev)
        for side in sides:
            x0, y0 = int(rng.integers(0, qm.W - side + 1)), int(rng.integers(0, qm.H - side + 1))
            t = (q64[y0:y0 + side, x0:x0 + side]
                 + 0.05 * rng.standard_normal((side, side, qm.D))).astype(np.float32)
            seed = len(pairs) + 1
            tp = B.vqnnf_codebook(ctx, t, k, 20, seed, B.default_bank(side, side, 3))
            heat = torch.full(((qm.H - side + 1) * (qm.W - side + 1),), float("nan"), device="cuda")
            pairs.append((tp, B.device_fmap(dev, qm.dtype), heat, q64, t.astype(np.float64), k, side, side, seed))

    add_float_map(synth.random_map(70, 90, 64, "f32", seed=71, M=20), (14, 20), 16)
    add_float_map(synth.random_map(60, 75, 18, "f32", seed=72, M=16), (12,), 32)
    add_float_map(synth.random_map(64, 80, 128, "bf16", seed=73, M=20), (16, 24), 32)
    img = synth.rgb_image(72, 96, seed=74)
    dimg = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    devs.append(dimg)
    qf = O.rgb_patch_features(img)
    for tw, th in ((18, 16), (24, 24)):
        x0, y0 = int(rng.integers(0, 96 - tw + 1)), int(rng.integers(0, 72 - th + 1))
        crop = np.ascontiguousarray(img[y0:y0 + th, x0:x0 + tw])
        seed = len(pairs) + 1
        tp = B.vqnnf_codebook(ctx, crop, 24, 20, seed, B.default_bank(tw, th, 3))
        heat = torch.full(((72 - th + 1) * (96 - tw + 1),), float("nan"), device="cuda")
        pairs.append((tp, B.device_fmap(dimg, "rgb8"), heat, qf, O.rgb_patch_features(crop), 24, tw, th, seed))
    tpls = [p[0] for p in pairs]
    fms = [p[1] for p in pairs]
    heats = [p[2] for p in pairs]
    log(f"mixed batch: {len(pairs)} pairs over FP32, low-D FP32, BF16 and RGB maps")
    out = B.vqnnf_match_batched(ctx, tpls, fms, P, heats)
    refs, bests = per_pair(ctx, tpls, fms, heats, P)
    for i in range(len(pairs)):
        assert torch.equal(heats[i], refs[i]), f"pair {i}"
        assert out[i] == bests[i], f"pair {i}: {out[i]} vs {bests[i]}"
    for i in (0, 2, len(pairs) - 1):
        tp, _, heat, qx, tx, k, w, h, seed = pairs[i]
        cb32 = O.kmeans_codebook(tx.astype(np.float32), k, 20, seed)
        assert np.array_equal(tp.codebook().view(np.uint32), cb32.view(np.uint32)), f"pair {i} codebook"
        cb = cb32.astype(np.float64)
        filters = O.expand_bank(O.default_bank(w, h, 3))
        rt = O.template_representation(O.assign_map(tx, cb), k, filters)
        sim = O.similarity_map_fast(O.assign_map(qx, cb), k, w, h, filters, rt)
        gpu = heat.cpu().numpy().reshape(sim.shape).astype(np.float64)
        err = np.abs(gpu - sim)
        log(f"pair {i} vs oracle: max abs err {err.max():.3e}")
        assert (err <= REL * np.abs(sim) + ABS).all(), f"pair {i}"
