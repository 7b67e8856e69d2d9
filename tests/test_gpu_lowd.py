"""Low-dimensional features (D <= 32, F32 / BF16) and RGB colour features
built on the GPU (3x3 patches, D = 27) through the C ABI: labels bit-exact
against the FP64 oracle, exact ties resolved to the lower index, the colour
templates' k-means bit-identical to the oracle's, and the matching heatmap on
RGB images within the parity tolerance with the planted crop found."""
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


@pytest.mark.parametrize("H,W,D,dt,k,seed", [(120, 150, 9, "f32", 16, 1), (97, 131, 18, "f32", 128, 2),
                                             (64, 77, 27, "f32", 256, 3), (50, 61, 32, "f32", 64, 4),
                                             (88, 90, 18, "bf16", 128, 5), (40, 45, 9, "bf16", 7, 6),
                                             (33, 35, 1, "f32", 12, 7)])
def test_lowd_assign_bit_exact(ctx, H, W, D, dt, k, seed):
    log(f"low-D assign {H}x{W} D={D} {dt} k={k}")
    qm = synth.random_map(H, W, D, dt, seed=seed, M=max(4, k // 2))
    q64 = O.decode(qm.dtype, qm.data, qm.scale)
    rng = np.random.default_rng(seed)
    src = q64.reshape(-1, D)
    cb = (src[rng.integers(0, len(src), size=k)] + 0.05 * rng.standard_normal((k, D))).astype(np.float32)
    tmpl = q64[:8, :8].astype(np.float32)
    tpl = B.vqnnf_template_from_codebook(ctx, tmpl, cb, B.default_bank(8, 8, 1))
    lab = torch.empty(H * W, dtype=torch.uint8, device="cuda")
    nf = B.vqnnf_assign(ctx, tpl, B.device_fmap(to_dev(qm), dt), B.VQNNF_PREC_BF16_REFINED, lab)
    ref = O.assign(src, cb.astype(np.float64))
    got = lab.cpu().numpy().astype(np.int64)
    log(f"  flagged {nf}, mismatches {(got != ref).sum()}")
    assert np.array_equal(got, ref)
    B.vqnnf_assign(ctx, tpl, B.device_fmap(to_dev(qm), dt), B.VQNNF_PREC_FP32_PLAIN, lab)
    assert int((lab.cpu().numpy().astype(np.int64) != ref).sum()) <= max(2, H * W // 100)


def test_lowd_exact_ties_and_duplicates(ctx):
    rng = np.random.default_rng(12)
    for D in (9, 18, 27):
        k = 10
        cb = (rng.integers(-64, 64, size=(k, D)) / 32.0).astype(np.float32)
        cb[6] = cb[1]
        pts = [(cb[a].astype(np.float64) + cb[b]) / 2
               for a, b in (sorted(rng.choice(k, size=2, replace=False)) for _ in range(500))]
        pts += [cb[j].astype(np.float64) for j in range(k)]
        q = np.array(pts, dtype=np.float32).reshape(1, -1, D)
        n = q.shape[1]
        tpl = B.vqnnf_template_from_codebook(ctx, q[:, :4].reshape(1, 4, D), cb, [(0, 0, 4, 1, 1, 1, 1.0)])
        lab = torch.empty(n, dtype=torch.uint8, device="cuda")
        nf = B.vqnnf_assign(ctx, tpl, B.device_fmap(torch.from_numpy(q).cuda(), "f32"),
                            B.VQNNF_PREC_BF16_REFINED, lab)
        x = q.reshape(n, D).astype(np.float64)
        ref = O.assign(x, cb.astype(np.float64))
        d = np.sort(O.sq_distances(x, cb.astype(np.float64)), axis=1)
        ties = int((d[:, 0] == d[:, 1]).sum())     # exact FP64 ties between the two nearest
        got = lab.cpu().numpy().astype(np.int64)
        log(f"ties D={D}: {ties} exact top-2 ties, flagged {nf}, mismatches {(got != ref).sum()}")
        assert ties >= 100 and nf >= ties
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("H,W,tw,th,k,stride", [(160, 200, 40, 36, 32, 3), (97, 130, 25, 31, 64, 4)])
def test_rgb_colour_features(ctx, H, W, tw, th, k, stride):
    img = synth.rgb_image(H, W, seed=H + W)
    rng = np.random.default_rng(W)
    x0, y0 = int(rng.integers(0, W - tw + 1)), int(rng.integers(0, H - th + 1))
    crop = np.ascontiguousarray(img[y0:y0 + th, x0:x0 + tw])
    bank = B.default_bank(tw, th, 3)
    log(f"RGB {H}x{W} (pixel stride {stride}), template {tw}x{th}, k={k}")
    tpl = B.vqnnf_codebook(ctx, crop, k, 20, 3, bank)
    # the template's colour features and k-means, by the oracle
    tf = O.rgb_patch_features(crop)
    ref_cb = O.kmeans_codebook(tf.astype(np.float32), k, 20, 3)
    assert np.array_equal(tpl.codebook().view(np.uint32), ref_cb.view(np.uint32))
    padded = np.zeros((H, W, stride), np.uint8)
    padded[:, :, :3] = img
    padded[:, :, 3:] = 77                       # padding bytes are never read as colour
    d = torch.from_numpy(padded).cuda()
    fm = B.device_fmap(d, "rgb8")
    lab = torch.empty(H * W, dtype=torch.uint8, device="cuda")
    nf = B.vqnnf_assign(ctx, tpl, fm, B.VQNNF_PREC_BF16_REFINED, lab)
    qf = O.rgb_patch_features(img)
    ql = O.assign_map(qf, ref_cb.astype(np.float64))
    got = lab.cpu().numpy().astype(np.int64).reshape(H, W)
    log(f"  flagged {nf}, label mismatches {(got != ql).sum()}")
    assert np.array_equal(got, ql)
    heat = torch.full(((H - th + 1) * (W - tw + 1),), float("nan"), device="cuda")
    (bx, by), _ = B.vqnnf_match(ctx, tpl, fm, B.VQNNF_PREC_BF16_REFINED, heat)
    filters = O.expand_bank(O.default_bank(tw, th, 3))
    tl = O.assign_map(tf, ref_cb.astype(np.float64))
    sim = O.similarity_map_fast(ql, k, tw, th, filters, O.template_representation(tl, k, filters))
    g = heat.cpu().numpy().astype(np.float64).reshape(sim.shape)
    err = np.abs(g - sim)
    log(f"  heatmap max abs err {err.max():.3e}; best ({bx}, {by}), planted ({x0}, {y0})")
    assert (err <= REL * np.abs(sim) + ABS).all()
    assert (bx, by) == (x0, y0)
