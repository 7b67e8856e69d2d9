"""Full-size parity of the three benchmark workloads against the oracle's
stored results (tests/golden/fullsize_labels.json and c3_query_labels.npz,
written by tests/golden/make_fullsize_golden.py from the oracle alone).

For every (template, map) pair, at the full map sizes and in the launch
configurations the benchmark times:
  * the generator reproduces the inputs the oracle saw (template and map
    hashes);
  * the library's k-means (on the GPU) reproduces the oracle's codebook
    (hash of the FP32 codebook);
  * the label map of the refined path equals the oracle's exact FP64
    nearest-codeword map bit for bit (Alg. 1; Sec. 5.2 "exact NN"): the
    single-pair call (vqnnf_assign) and, for the batched workloads, the
    label maps the fused batched call computed (vqnnf_batched_labels);
  * c3 (1024x1024, D=512 BF16, k=128): every one of the 863041 heatmap
    values of vqnnf_match against the oracle's eq. 2 on its own labels, to
    1e-5 relative plus 2^-24 * S_max (S_max = 4), and the best window;
  * c4 (64 templates on one 1024x1024 D=256 map) and c5 (32 FP8 maps with
    sides 256..2048, 4 templates each): the batched heatmaps (graph mode)
    equal the single-pair path's bit for bit.
The c5 maps are generated in four tests of eight maps each (the generator
makes each map from its own streams), then matched as one batch."""
import hashlib
import json
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from oracle import vqnnf_oracle as O
from paper_2306_15010_amd import binding as B
from paper_2306_15010_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
REL, ABS = 1e-5, 4 * 2.0 ** -24
P = B.VQNNF_PREC_BF16_REFINED

with open(os.path.join(HERE, "golden", "fullsize_labels.json")) as _f:
    GOLD = json.load(_f)


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def _dev(qm):
    if qm.dtype == "bf16":
        return torch.from_numpy(qm.data.view(np.int16)).cuda()
    return torch.from_numpy(np.ascontiguousarray(qm.data)).cuda()


def _check_inputs(qm, row, gmap):
    assert (qm.H, qm.W, qm.D, qm.dtype) == (gmap["H"], gmap["W"], gmap["D"], gmap["dtype"])
    assert sha(qm.data) == gmap["map_sha256"], "generator output changed: rerun make_fullsize_golden.py"
    if qm.scale is not None:
        assert sha(qm.scale) == gmap["scale_sha256"]
    assert len(row) == len(gmap["pairs"])
    for t, g in zip(row, gmap["pairs"]):
        assert sha(t.data.astype(np.float32)) == g["template_sha256"]
        assert (t.k, t.x0, t.y0) == (g["k"], g["x0"], g["y0"])


def _gpu_sha(lab):
    torch.cuda.synchronize()
    return sha(lab.cpu().numpy())


def _oracle_heatmap_bands(labels, k, w, h, filters, rt, band=64):
    """Eq. 2 for every window, from row bands of the label map (a window
    depends only on the labels inside it), bands on a few threads."""
    H, W = labels.shape
    oh = H - h + 1
    starts = list(range(0, oh, band))

    def one(y0):
        y1 = min(oh, y0 + band)
        return y0, O.similarity_map_fast(labels[y0:y1 + h - 1], k, w, h, filters, rt)

    out = np.empty((oh, W - w + 1))
    with ThreadPoolExecutor(max_workers=min(8, len(os.sched_getaffinity(0)))) as ex:
        for y0, sim in ex.map(one, starts):
            out[y0:y0 + sim.shape[0]] = sim
    return out


# ------------------------------------------------------------------ c3

def test_c3_full_labels_and_heatmap():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g = GOLD["c3"]["maps"][0]
    log("generating the 1024x1024 D=512 BF16 workload")
    wl = synth.make_config("c3")
    qm, t = wl.maps[0], wl.templates[0][0]
    _check_inputs(qm, [t], g)
    gp = g["pairs"][0]
    ctx = B.Context(stream=torch.cuda.current_stream())
    tpl = B.vqnnf_codebook(ctx, t.data, t.k, 20, gp["seed"], B.default_bank(96, 96, 3))
    assert sha(tpl.codebook()) == gp["codebook_sha256"]
    qd = _dev(qm)
    fm = B.device_fmap(qd, "bf16")
    H, W = qm.H, qm.W
    lab = torch.empty(H * W, dtype=torch.uint8, device="cuda")
    nflag = B.vqnnf_assign(ctx, tpl, fm, P, lab)
    gl = np.load(os.path.join(HERE, "golden", "c3_query_labels.npz"))["labels"]
    assert sha(gl) == gp["labels_sha256"]
    got = lab.cpu().numpy().reshape(H, W)
    log(f"flagged {nflag}; label mismatches vs the oracle: {int((got != gl).sum())} of {H * W}")
    assert np.array_equal(got, gl)
    # the benchmark's call: vqnnf_match on the same pair
    oh, ow = H - 95, W - 95
    heat = torch.full((oh * ow,), float("nan"), device="cuda")
    (bx, by), bs = B.vqnnf_match(ctx, tpl, fm, P, heat)
    hm = heat.cpu().numpy().reshape(oh, ow).astype(np.float64)
    log("oracle heatmap of all windows from the oracle's labels")
    filters = O.expand_bank(O.default_bank(96, 96, 3))
    cb64 = tpl.codebook().astype(np.float64)
    tl = O.assign_map(t.data.astype(np.float64), cb64)
    rt = O.template_representation(tl, t.k, filters)
    ref = _oracle_heatmap_bands(gl.astype(np.int64), t.k, 96, 96, filters, rt)
    err = np.abs(hm - ref)
    bad = err > REL * np.abs(ref) + ABS
    log(f"heatmap: {ref.size} windows, max abs err {err.max():.3e}, max rel {np.max(err / np.maximum(np.abs(ref), 1e-30)):.3e}")
    assert not bad.any(), f"{int(bad.sum())} windows outside tolerance"
    i = int(np.argmax(hm.reshape(-1)))
    assert (bx, by) == (i % ow, i // ow)
    # the oracle's own best window scores the same within tolerance
    ox, oy, os_ = O.localise(ref)
    assert abs(ref[by, bx] - os_) <= REL * abs(os_) + 2 * ABS
    log(f"best {(bx, by)} (oracle {(ox, oy)}), planted {(t.x0, t.y0)}")
    ctx.close()


# ------------------------------------------------------------------ c4 / c5

def _batched_full(ctx, maps, rows, gmaps, seed0):
    """Codebooks (GPU k-means, batched), single-pair labels, then the whole
    batch in graph mode: its label maps and heatmaps."""
    tmpls, ks, seeds, banks, pairs = [], [], [], [], []
    for mi, (qm, row, gm) in enumerate(zip(maps, rows, gmaps)):
        _check_inputs(qm, row, gm)
        for t, gp in zip(row, gm["pairs"]):
            h, w, _ = t.data.shape
            tmpls.append(t.data)
            ks.append(t.k)
            seeds.append(gp["seed"])
            banks.append(B.default_bank(w, h, t.grid))
            pairs.append((mi, t, gp))
    assert seeds == list(range(seed0, seed0 + len(seeds)))
    log(f"k-means of {len(tmpls)} templates on the GPU (one batched call)")
    tpls = B.vqnnf_codebook_batched(ctx, tmpls, ks, 20, seeds, banks)
    for tpl, (_, _, gp) in zip(tpls, pairs):
        assert sha(tpl.codebook()) == gp["codebook_sha256"]
    devs = [_dev(qm) for qm in maps]
    fms = [B.device_fmap(d, qm.dtype, qm.scale) for d, qm in zip(devs, maps)]
    # single-pair labels
    for i, (tpl, (mi, t, gp)) in enumerate(zip(tpls, pairs)):
        qm = maps[mi]
        lab = torch.empty(qm.H * qm.W, dtype=torch.uint8, device="cuda")
        B.vqnnf_assign(ctx, tpl, fms[mi], P, lab)
        assert _gpu_sha(lab) == gp["labels_sha256"], f"pair {i}: single-pair labels differ from the oracle"
    log(f"{len(pairs)} single-pair label maps equal the oracle's")
    # the batch, captured as a graph and replayed
    heats = [torch.full(((maps[mi].H - t.data.shape[0] + 1) * (maps[mi].W - t.data.shape[1] + 1),),
                        float("nan"), device="cuda") for (mi, t, _) in pairs]
    qlist = [fms[mi] for (mi, _, _) in pairs]
    B.vqnnf_ctx_set_graph(ctx, True)
    try:
        B.vqnnf_match_batched(ctx, tpls, qlist, P, heats, want_best=False)
        out = B.vqnnf_match_batched(ctx, tpls, qlist, P, heats)
    finally:
        B.vqnnf_ctx_set_graph(ctx, False)
    for i, (mi, t, gp) in enumerate(pairs):
        qm = maps[mi]
        lab = torch.empty(qm.H * qm.W, dtype=torch.uint8, device="cuda")
        B.vqnnf_batched_labels(ctx, i, lab)
        assert _gpu_sha(lab) == gp["labels_sha256"], f"pair {i}: batched labels differ from the oracle"
    log(f"{len(pairs)} batched label maps equal the oracle's")
    found = 0
    for i, (tpl, (mi, t, gp)) in enumerate(zip(tpls, pairs)):
        ref = torch.empty_like(heats[i])
        best = B.vqnnf_match(ctx, tpl, fms[mi], P, ref)
        assert torch.equal(heats[i], ref), f"pair {i}: batched heatmap differs from vqnnf_match"
        assert out[i] == best
        found += best[0] == (t.x0, t.y0)
    log(f"batched heatmaps equal the single-pair path; planted crop best for {found} of {len(pairs)}")
    torch.cuda.synchronize()
    for tpl in tpls:
        tpl.free()


def test_c4_full_labels_single_and_batched():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    log("generating the 64-template 1024x1024 D=256 BF16 workload")
    wl = synth.make_config("c4")
    ctx = B.Context(stream=torch.cuda.current_stream())
    _batched_full(ctx, wl.maps, wl.templates, GOLD["c4"]["maps"], 0)
    ctx.close()


_C5 = {}


@pytest.mark.parametrize("part", range(4))
def test_c5_generate_full_size(part):
    """Makes maps 8*part .. 8*part+7 of the 32-map FP8 workload at full size
    (checked against the stored hashes) for the batched test below."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    idx = list(range(8 * part, 8 * part + 8))
    wl = synth.make_config("c5", maps=idx)
    for i, qm, row in zip(idx, wl.maps, wl.templates):
        _check_inputs(qm, row, GOLD["c5"]["maps"][i])
        _C5[i] = (qm, row)
    log(f"maps {idx[0]}..{idx[-1]} made: {[(qm.W, qm.H) for qm in wl.maps]}")


def test_c5_full_labels_single_and_batched():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if len(_C5) != 32:
        pytest.skip("the c5 maps were not generated (run the whole module)")
    maps = [_C5[i][0] for i in range(32)]
    rows = [_C5[i][1] for i in range(32)]
    ctx = B.Context(stream=torch.cuda.current_stream())
    _batched_full(ctx, maps, rows, GOLD["c5"]["maps"], 0)
    ctx.close()
    _C5.clear()
