"""FP8 (E4M3FN codes x per-channel FP32 scale) query maps on the GPU.

The stored codes times their scale are the query values (exact in FP64);
the refined path must label every pixel exactly as the FP64 oracle does, on
the fast path (D a multiple of 64, aligned rows) and the bounds-checked one,
and the whole match must agree with the oracle's heatmap.  The scale is
folded into a per-scale copy of the codebook, so two maps with different
scales against one template exercise two such copies."""
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


def fp8_map(H, W, D, seed, M=24, zero_channel=None):
    rng = np.random.default_rng(seed)
    means = rng.standard_normal((M, D))
    z = synth.smooth_label_field(H, W, M, rng)
    q = synth.mixture_features(z, means, 0.3, rng)
    if zero_channel is not None:
        q[..., zero_channel] = 0.0
    return synth.encode(q, "fp8")


@pytest.mark.parametrize("H,W,D,k,seed", [
    (48, 56, 64, 16, 1),      # fast path
    (40, 45, 256, 64, 2),     # fast path, c5 shape
    (33, 37, 100, 32, 3),     # bounds-checked path (D not a multiple of 64)
    (29, 31, 128, 128, 4),
    (20, 23, 27, 5, 5),
])
def test_fp8_assign_exact(ctx, H, W, D, k, seed):
    qm = fp8_map(H, W, D, seed, zero_channel=D // 3)
    assert qm.scale[D // 3] == 1.0   # an all-zero channel keeps scale 1 (codes 0)
    q = qm.decoded_f32()
    rng = np.random.default_rng(seed + 100)
    ys, xs = rng.integers(0, H - 8), rng.integers(0, W - 8)
    t = np.ascontiguousarray(q[ys:ys + 8, xs:xs + 8].astype(np.float32))
    tpl = B.vqnnf_codebook(ctx, t, k, 10, seed, B.default_bank(8, 8, 2))
    dev = torch.from_numpy(qm.data).cuda()
    fm = B.device_fmap(dev, "fp8", qm.scale)
    lab = torch.empty(H * W, dtype=torch.uint8, device="cuda")
    log(f"fp8 assign {H}x{W} D={D} k={k}")
    nfl = B.vqnnf_assign(ctx, tpl, fm, B.VQNNF_PREC_BF16_REFINED, lab)
    cb32 = O.kmeans_codebook(t, k, 10, seed)
    assert np.array_equal(tpl.codebook().view(np.uint32), cb32.view(np.uint32))
    ref = O.assign_map(O.decode("fp8", qm.data, qm.scale), cb32.astype(np.float64))
    got = lab.cpu().numpy().reshape(H, W).astype(np.int64)
    log(f"  flagged {nfl}, mismatches {(got != ref).sum()}")
    assert np.array_equal(got, ref)
    # the plain path: FP32 products of the exact codes with the rounded s*c
    B.vqnnf_assign(ctx, tpl, fm, B.VQNNF_PREC_FP32_PLAIN, lab)
    mism = int((lab.cpu().numpy().reshape(H, W) != ref).sum())
    log(f"  plain FP32 mismatches {mism}")
    assert mism <= max(2, H * W // 200)


def test_fp8_match_and_two_scales(ctx):
    wl = synth.make_multi_map(61, 2, (64, 128), 64, 32, 0.3, "fp8", 2, (16, 32), 32, 3)
    assert not np.array_equal(wl.maps[0].scale, wl.maps[1].scale)
    # the first map's first template matched against both maps: two scaled copies
    t0 = wl.templates[0][0]
    h, w, _ = t0.data.shape
    tpl = B.vqnnf_codebook(ctx, t0.data, t0.k, 20, 0, B.default_bank(w, h, 3))
    filters = O.expand_bank(O.default_bank(w, h, 3))
    cb32 = O.kmeans_codebook(t0.data, t0.k, 20, 0)
    assert np.array_equal(tpl.codebook().view(np.uint32), cb32.view(np.uint32))
    cb = cb32.astype(np.float64)
    rt = O.template_representation(O.assign_map(t0.data.astype(np.float64), cb), t0.k, filters)
    for mi, qm in enumerate(wl.maps):
        dev = torch.from_numpy(qm.data).cuda()
        fm = B.device_fmap(dev, "fp8", qm.scale)
        heat = torch.full(((qm.H - h + 1) * (qm.W - w + 1),), float("nan"), device="cuda")
        (bx, by), bs = B.vqnnf_match(ctx, tpl, fm, B.VQNNF_PREC_BF16_REFINED, heat)
        labels = O.assign_map(O.decode("fp8", qm.data, qm.scale), cb)
        sim = O.similarity_map_fast(labels, t0.k, w, h, filters, rt)
        gpu = heat.cpu().numpy().reshape(sim.shape).astype(np.float64)
        err = np.abs(gpu - sim)
        log(f"map {mi} {qm.H}x{qm.W}: max err {err.max():.3e}, best {(bx, by)}")
        assert (err <= REL * np.abs(sim) + ABS).all()
        i = int(np.argmax(gpu.reshape(-1)))
        assert (bx, by) == (i % sim.shape[1], i // sim.shape[1])
        if mi == 0:
            assert (bx, by) == (t0.x0, t0.y0)


def test_fp8_batched_graph_scale_change(ctx):
    wl = synth.make_multi_map(67, 2, (64, 128), 64, 32, 0.3, "fp8", 2, (16, 32), 16, 2)
    tpls, fms, heats, devs = [], [], [], []
    for qm, row in zip(wl.maps, wl.templates):
        dev = torch.from_numpy(qm.data).cuda()
        devs.append(dev)
        for t in row:
            h, w, _ = t.data.shape
            tpls.append(B.vqnnf_codebook(ctx, t.data, t.k, 20, 0, B.default_bank(w, h, t.grid)))
            fms.append(B.device_fmap(dev, "fp8", qm.scale))
            heats.append(torch.empty((qm.H - h + 1) * (qm.W - w + 1), device="cuda"))
    P = B.VQNNF_PREC_BF16_REFINED
    eager = B.vqnnf_match_batched(ctx, tpls, fms, P, heats)
    refs = [h.clone() for h in heats]
    B.vqnnf_ctx_set_graph(ctx, True)
    try:
        for rep in range(2):
            out = B.vqnnf_match_batched(ctx, tpls, fms, P, heats)
            assert out == eager
            assert all(torch.equal(a, b) for a, b in zip(heats, refs))
        # same pointers, new scale values for map 0: different tables, new capture
        s2 = (wl.maps[0].scale * np.float32(1.5)).astype(np.float32)
        for i in range(2):
            fms[i]._scale[:] = s2
        out2 = B.vqnnf_match_batched(ctx, tpls, fms, P, heats)
    finally:
        B.vqnnf_ctx_set_graph(ctx, False)
    for i in range(len(tpls)):
        r = torch.empty_like(heats[i])
        assert B.vqnnf_match(ctx, tpls[i], fms[i], P, r) == out2[i]
        assert torch.equal(r, heats[i]), i


def test_fp8_precision_enum_same_results(ctx):
    """VQNNF_PREC_FP8_REFINED on an FP8 map runs the refined search: the same
    labels, heatmap and best window as VQNNF_PREC_BF16_REFINED, in single and
    batched calls; the labels are the oracle's."""
    qm = fp8_map(64, 72, 64, 9)
    q = qm.decoded_f32()
    t = np.ascontiguousarray(q[10:26, 20:36].astype(np.float32))
    tpl = B.vqnnf_codebook(ctx, t, 16, 20, 2, B.default_bank(16, 16, 2))
    dev = torch.from_numpy(qm.data).cuda()
    fm = B.device_fmap(dev, "fp8", qm.scale)
    la = torch.empty(64 * 72, dtype=torch.uint8, device="cuda")
    lb = torch.empty_like(la)
    B.vqnnf_assign(ctx, tpl, fm, B.VQNNF_PREC_BF16_REFINED, la)
    B.vqnnf_assign(ctx, tpl, fm, B.VQNNF_PREC_FP8_REFINED, lb)
    assert torch.equal(la, lb)
    cb32 = O.kmeans_codebook(t, 16, 20, 2)
    assert np.array_equal(tpl.codebook().view(np.uint32), cb32.view(np.uint32))
    ref = O.assign_map(O.decode("fp8", qm.data, qm.scale), cb32.astype(np.float64))
    assert np.array_equal(lb.cpu().numpy().reshape(64, 72).astype(np.int64), ref)
    ha = torch.full((49 * 57,), float("nan"), device="cuda")
    hb = torch.full_like(ha, float("nan"))
    ba = B.vqnnf_match(ctx, tpl, fm, B.VQNNF_PREC_BF16_REFINED, ha)
    bb = B.vqnnf_match(ctx, tpl, fm, B.VQNNF_PREC_FP8_REFINED, hb)
    assert ba == bb and torch.equal(ha, hb)
    hc = torch.full_like(ha, float("nan"))
    out = B.vqnnf_match_batched(ctx, [tpl], [fm], B.VQNNF_PREC_FP8_REFINED, [hc])
    assert out[0] == ba and torch.equal(ha, hc)
    log(f"FP8 precision enum: best {bb}")
