"""Full-size parity of batched matching on the 64-template workload: one
1024x1024 BF16 map with D = 256 and 64 templates (sides 24..160, k in
{16, 32, 64, 128}, full window + 2x2 grid), in the launch configuration the
benchmark times (all 64 pairs in one vqnnf_match_batched call, captured as a
HIP graph and replayed).

The codebooks are drawn without the library (template pixels plus seeded
jitter; the library's k-means is pinned bit for bit elsewhere), so the oracle
needs no k-means of 64 templates.  It cannot label the whole map for 64
codebooks in seconds, so it checks:
  * for the three cheapest templates of every codebook size and for the
    largest template, the heatmap at the planted window and at a random
    window, from the oracle's own labels of those windows' pixels, to the
    parity tolerance;
  * for every pair, that the reported best is the first maximum of its
    heatmap, and that the graph replay reproduces the captured call.
Every pair's heatmap must also equal, bit for bit, the one vqnnf_match gives
for that pair alone (that path is pinned to the oracle at full size)."""
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


def test_c4_batched_full_size():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    log("generating the 64-template 1024x1024 D=256 workload")
    wl = synth.make_config("c4")
    qm, row = wl.maps[0], wl.templates[0]
    H, W, D = qm.H, qm.W, qm.D
    ctx = B.Context(stream=torch.cuda.current_stream())
    rng = np.random.default_rng(4064)
    cbs, tpls, heats = [], [], []
    dev = torch.from_numpy(qm.data.view(np.int16)).cuda()
    fm = B.device_fmap(dev, "bf16")
    for t in row:
        h, w, _ = t.data.shape
        src = t.data.reshape(-1, D)
        cb = (src[rng.integers(0, len(src), size=t.k)]
              + 0.05 * rng.standard_normal((t.k, D))).astype(np.float32)
        cbs.append(cb)
        tpls.append(B.vqnnf_template_from_codebook(ctx, t.data, cb, B.default_bank(w, h, t.grid)))
        heats.append(torch.full(((H - h + 1) * (W - w + 1),), float("nan"), device="cuda"))
    P = B.VQNNF_PREC_BF16_REFINED
    n = len(row)
    log(f"{n} pairs; batched call in graph mode (capture, then replay)")
    B.vqnnf_ctx_set_graph(ctx, True)
    try:
        out = B.vqnnf_match_batched(ctx, tpls, [fm] * n, P, heats)
        first = [h.clone() for h in heats]
        for h in heats:
            h.fill_(float("nan"))
        out2 = B.vqnnf_match_batched(ctx, tpls, [fm] * n, P, heats)
        torch.cuda.synchronize()
    finally:
        B.vqnnf_ctx_set_graph(ctx, False)
    assert out2 == out
    for i in range(n):
        assert torch.equal(heats[i], first[i]), f"replay, pair {i}"
    del first
    # every pair against the single-pair path, and the best as the first maximum
    found = 0
    for i, t in enumerate(row):
        h, w, _ = t.data.shape
        ow = W - w + 1
        ref = torch.empty_like(heats[i])
        best = B.vqnnf_match(ctx, tpls[i], fm, P, ref)
        assert torch.equal(heats[i], ref), f"pair {i} differs from vqnnf_match"
        assert out[i] == best, (i, out[i], best)
        j = int(torch.argmax(heats[i]).item())
        (bx, by), bs = out[i]
        assert (bx, by) == (j % ow, j // ow) and bs == float(heats[i][j].item()), i
        found += (bx, by) == (t.x0, t.y0)
    log(f"planted crop is the best window for {found} of {n} pairs")
    # the oracle on sampled windows
    picks = []
    for k in sorted({t.k for t in row}):
        idx = sorted((i for i, t in enumerate(row) if t.k == k), key=lambda i: row[i].data.shape[0])
        picks += idx[:3]
    picks.append(max(range(n), key=lambda i: row[i].data.shape[0]))
    for i in picks:
        t = row[i]
        h, w, _ = t.data.shape
        oh, ow = H - h + 1, W - w + 1
        cb64 = cbs[i].astype(np.float64)
        filters = O.expand_bank(O.default_bank(w, h, t.grid))
        tl = O.assign_map(t.data.astype(np.float64), cb64)
        assert np.array_equal(tpls[i].labels().astype(np.int64), tl)
        rt = O.template_representation(tl, t.k, filters)
        hm = heats[i].cpu().numpy()
        wins = [(t.x0, t.y0), (int(rng.integers(0, ow)), int(rng.integers(0, oh)))]
        for (x, y) in wins:
            ql = O.assign_map(O.decode("bf16", qm.data[y:y + h, x:x + w]), cb64)
            sim = O.similarity_map_fast(ql, t.k, w, h, filters, rt)
            assert sim.shape == (1, 1)
            ref, got = float(sim[0, 0]), float(hm[y * ow + x])
            log(f"pair {i} ({w}x{h}, k={t.k}) window ({x},{y}): oracle {ref:.6g} gpu {got:.6g}")
            assert abs(got - ref) <= REL * abs(ref) + ABS, (i, x, y, got, ref)
    torch.cuda.synchronize()
    ctx.close()
