"""PCA reduction on the GPU (vqnnf_pca_project) and the low-dimensional
matching path it feeds (Sec. 5.5).

Projection tolerance, derived (u = 2^-24, first order, the test allows twice
the bound):
  * FP32 / FP8 / RGB maps: an FMA chain over the D terms (q_t - m_t) * b_t with
    the subtraction rounded (FP8 values also rounded once when decoded), so
    |gpu - exact| <= (D + 3) u sum_t |q_t - m_t| |b_t|;
  * BF16 maps on the matrix cores: exact products of the BF16 elements with the
    three exact BF16 terms of each basis value, about 3D FP32 additions, then
    minus mean . basis (rounded once), so
    |gpu - exact| <= (3D + 4) u sum_t (|q_t| + |m_t|) |b_t|."""
import sys

import numpy as np
import pytest

from oracle import vqnnf_oracle as O
from paper_2306_15010_amd import binding as B
from paper_2306_15010_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = 2.0 ** -24
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


def dev(qm):
    if qm.dtype == "f32":
        return torch.from_numpy(np.ascontiguousarray(qm.data)).cuda()
    if qm.dtype == "bf16":
        return torch.from_numpy(qm.data.view(np.int16)).cuda()
    return torch.from_numpy(np.ascontiguousarray(qm.data)).cuda()


@pytest.mark.parametrize("H,W,D,dt,d", [(150, 170, 256, "bf16", 18), (97, 103, 64, "f32", 9),
                                        (80, 90, 128, "fp8", 18), (120, 110, 27, "rgb8", 9),
                                        (33, 40, 512, "bf16", 64)])
def test_projection_parity(ctx, H, W, D, dt, d):
    if dt == "rgb8":
        img = synth.rgb_image(H, W, seed=7)
        x = O.rgb_patch_features(img)
        fm = B.device_fmap(torch.from_numpy(img).cuda(), "rgb8")
        tmpl = img[:30, :30].copy()
    else:
        qm = synth.random_map(H, W, D, dt, seed=H, M=24)
        x = O.decode(qm.dtype, qm.data, qm.scale)
        fm = B.device_fmap(dev(qm), dt, qm.scale)
        tmpl = x[:30, :30].astype(np.float32)
    # the oracle's own PCA of the template, rounded to FP32 (the arguments the
    # projection takes)
    om, ob, _ = O.pca_fit(tmpl.reshape(-1, D).astype(np.float64), d)
    mean, basis = om.astype(np.float32), ob.astype(np.float32)
    out = torch.empty((H, W, d), dtype=torch.float32, device="cuda")
    B.vqnnf_pca_project(ctx, fm, mean, basis, out)
    xc = x.reshape(-1, D) - mean.astype(np.float64)
    ref = xc @ basis.astype(np.float64).T
    ab = np.abs(basis.astype(np.float64)).T
    if dt == "bf16":
        bound = 2 * (3 * D + 4) * U * ((np.abs(x.reshape(-1, D)) + np.abs(mean.astype(np.float64))) @ ab)
    else:
        bound = 2 * (D + 3) * U * (np.abs(xc) @ ab)
    got = out.cpu().numpy().reshape(-1, d).astype(np.float64)
    err = np.abs(got - ref)
    log(f"projection {H}x{W} D={D} {dt} -> {d}: max err {err.max():.3e}, max err/bound {(err / bound).max():.3f}")
    assert (err <= bound).all()


@pytest.mark.parametrize("d", [9, 18])
def test_low_d_match_end_to_end(ctx, d):
    """The matching path at D = d on PCA-reduced features.  The reduced
    template and query are the oracle's FP64 projections (its own PCA of the
    template) rounded to FP32; on them the library's k-means must equal the
    oracle's bit for bit, the labels must be exact and the heatmap within the
    parity tolerance.  The GPU projection of the same query stays within the
    projection bound of the oracle's, and matching on it finds the planted
    crop."""
    H, W, D, side, k = 256, 288, 256, 48, 32
    qm = synth.random_map(H, W, D, "bf16", seed=31, M=32)
    q64 = O.decode("bf16", qm.data)
    rng = np.random.default_rng(5)
    x0, y0 = int(rng.integers(0, W - side + 1)), int(rng.integers(0, H - side + 1))
    t = (q64[y0:y0 + side, x0:x0 + side] + 0.05 * rng.standard_normal((side, side, D))).astype(np.float32)
    om, ob, _ = O.pca_fit(t.reshape(-1, D).astype(np.float64), d)
    mean, basis = om.astype(np.float32), ob.astype(np.float32)
    t_low = O.pca_project(t.astype(np.float64), mean, basis).astype(np.float32)
    q_low = O.pca_project(q64, mean, basis).astype(np.float32)
    bank = B.default_bank(side, side, 3)
    tpl = B.vqnnf_codebook(ctx, t_low, k, 20, 0, bank)
    cb32 = O.kmeans_codebook(t_low, k, 20, 0)
    assert np.array_equal(tpl.codebook().view(np.uint32), cb32.view(np.uint32))
    cb = cb32.astype(np.float64)
    fm = B.device_fmap(torch.from_numpy(np.ascontiguousarray(q_low)).cuda(), "f32")
    lab = torch.empty(H * W, dtype=torch.uint8, device="cuda")
    nf = B.vqnnf_assign(ctx, tpl, fm, B.VQNNF_PREC_BF16_REFINED, lab)
    ql = O.assign_map(q_low.astype(np.float64), cb)
    assert np.array_equal(lab.cpu().numpy().reshape(H, W), ql.astype(np.uint8))
    heat = torch.full(((H - side + 1) * (W - side + 1),), float("nan"), device="cuda")
    (bx, by), _ = B.vqnnf_match(ctx, tpl, fm, B.VQNNF_PREC_BF16_REFINED, heat)
    filters = O.expand_bank(O.default_bank(side, side, 3))
    tl = O.assign_map(t_low.astype(np.float64), cb)
    sim = O.similarity_map_fast(ql, k, side, side, filters, O.template_representation(tl, k, filters))
    g = heat.cpu().numpy().astype(np.float64).reshape(sim.shape)
    log(f"low-D d={d}: flagged {nf}, heatmap max err {np.abs(g - sim).max():.3e}, best ({bx},{by}) planted ({x0},{y0})")
    assert (np.abs(g - sim) <= REL * np.abs(sim) + ABS).all()
    assert (bx, by) == (x0, y0)
    # the same query projected on the GPU, then matched
    qp = torch.empty((H, W, d), dtype=torch.float32, device="cuda")
    B.vqnnf_pca_project(ctx, B.device_fmap(dev(qm), "bf16"), mean, basis, qp)
    exact = O.pca_project(q64, mean, basis).reshape(-1, d)
    bound = 2 * (3 * D + 4) * U * ((np.abs(q64.reshape(-1, D)) + np.abs(mean.astype(np.float64)))
                                   @ np.abs(basis.astype(np.float64)).T)
    assert (np.abs(qp.cpu().numpy().reshape(-1, d).astype(np.float64) - exact) <= bound).all()
    heat2 = torch.full_like(heat, float("nan"))
    (bx2, by2), _ = B.vqnnf_match(ctx, tpl, B.device_fmap(qp, "f32"), B.VQNNF_PREC_BF16_REFINED, heat2)
    assert (bx2, by2) == (x0, y0)
