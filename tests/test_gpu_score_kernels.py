"""The on-chip score tile kernel at forced tile choices: 16- and 32-channel
blocks, several window rows per tile (1, odd, tall), in both accumulation
modes (sums of |T_j - C_j| with v_sad_u16 where every stored sum's bound,
twice its filters' area, fits 16 bits; sums of min(T_j, C_j) for larger
templates; the cases straddle that limit).

Eq. 2's L1 terms are exact integers in every mode and tile shape, and the
FP32 score of a window is formed from them by the same expression, so every
heatmap and best window must be bit-identical across the choices, and the
first one must match the FP64 oracle within the parity tolerance.  A tile
choice is forced through the tune file: a context reads the entry for the
shape and runs it without tuning (the file must come back unchanged, which
proves no tuning ran).  The batched path must equal the single-pair path
bit for bit with 16-channel blocks (untuned default) and with the last
candidate the tuner times (32-channel blocks)."""
import sys

import numpy as np
import pytest

from oracle import vqnnf_oracle as O
from paper_2306_15010_amd import binding as B
from paper_2306_15010_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL, ABS = 1e-5, 4 * 2.0 ** -24
WIDE = 65536          # tune-file flag of 32-channel tile blocks

CASES = [
    # H, W, w, h, g, k
    (64, 64, 16, 16, 2, 8),
    (100, 140, 25, 25, 3, 32),
    (150, 90, 48, 48, 3, 128),
    (60, 260, 33, 21, 4, 17),       # unequal bin widths: one sum per weight class
    (40, 40, 40, 40, 2, 5),         # a single window
    (129, 300, 30, 30, 1, 64),
    (96, 96, 96, 31, 3, 200),
    (120, 160, 40, 37, 3, 96),      # unequal band heights
    (240, 300, 250, 180, 3, 64),    # widest template: one tile column
    (300, 700, 96, 96, 3, 128),     # three tile columns, ragged last tile
    (90, 600, 17, 9, 4, 256),       # k = 256: sixteen channel groups
    (250, 250, 181, 181, 2, 32),    # twice the area 65522: |T - C| sums, at the limit
    (250, 250, 182, 181, 2, 32),    # twice the area 65884: min(T, C) sums
    (200, 260, 200, 170, 2, 64),    # min(T, C) sums, four channel groups
]
# (block width flag, window rows per tile; 0 = the default sizing); (0, 0)
# writes no entry: the untuned default
CHOICES = [(0, 0), (0, 1), (0, 5), (0, 64), (WIDE, 0), (WIDE, 1), (WIDE, 2), (WIDE, 7)]


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _labels(H, W, k, rng):
    coarse = rng.integers(0, k, size=(H // 3 + 2, W // 3 + 2))
    ql = np.kron(coarse, np.ones((3, 3), dtype=np.int64))[:H, :W]
    noise = rng.random((H, W)) < 0.3
    return np.where(noise, rng.integers(0, k, size=(H, W)), ql)


def _kpad(k):
    """Padded codebook size of the library: blocks of 16 codewords, rounded
    to 1, 2, 3, 4, 8 or 16 blocks."""
    kb = (k + 15) // 16
    kb = 8 if 4 < kb <= 8 else 16 if kb > 8 else kb
    return 16 * kb


def _n_cu():
    return torch.cuda.get_device_properties(0).multi_processor_count


@pytest.mark.parametrize("H,W,w,h,g,k", CASES)
def test_tile_kernels_agree_with_oracle(tmp_path, H, W, w, h, g, k):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(H * 31 + W * 7 + k)
    ql = _labels(H, W, k, rng)
    y0, x0 = int(rng.integers(0, H - h + 1)), int(rng.integers(0, W - w + 1))
    tl = ql[y0:y0 + h, x0:x0 + w]
    # one-hot codewords: the template's FP64 labels are exactly tl
    cb = np.eye(k, dtype=np.float32)
    tmpl = cb[tl]
    ld = torch.from_numpy(ql.astype(np.uint8).reshape(-1)).cuda()
    oh, ow = H - h + 1, W - w + 1
    kpad = _kpad(k)
    path = tmp_path / "tune.txt"
    outs = []
    for flag, tyw in CHOICES:
        # entries for both bin-weight classes of the key: only the template's
        # own is read
        text = "".join(f"s {_n_cu()} {w} {h} {g} {kpad} {H} {W} {u} {flag | tyw if flag | tyw else 1}\n"
                       for u in (0, 1))
        if flag == 0 and tyw == 0:
            text = ""   # no entry: the context tunes nothing (autotuning off) and uses the default
        path.write_text(text)
        ctx = B.Context(stream=torch.cuda.current_stream())
        if not text:
            B.vqnnf_ctx_set_autotune(ctx, 0)
        B.vqnnf_ctx_set_tune_file(ctx, path)
        tpl = B.vqnnf_template_from_codebook(ctx, tmpl, cb, B.default_bank(w, h, g))
        heat = torch.full((oh * ow,), float("nan"), device="cuda")
        best = B.vqnnf_score(ctx, tpl, ld, H, W, heat)
        torch.cuda.synchronize()
        assert path.read_text() == text, "the forced choice was not used (the context tuned)"
        outs.append((heat.cpu().numpy(), best))
        tpl.free()
        ctx.close()
    filters = O.expand_bank(O.default_bank(w, h, g))
    rt = O.template_representation(tl, k, filters)
    ref = O.similarity_map_fast(ql, k, w, h, filters, rt)
    hm = outs[0][0].reshape(oh, ow).astype(np.float64)
    err = np.abs(hm - ref)
    assert (err <= REL * np.abs(ref) + ABS).all(), f"max err {err.max():.3e}"
    assert outs[0][1][0] == O.localise(ref)[:2]
    for (flag, tyw), (hv, bv) in zip(CHOICES[1:], outs[1:]):
        name = f"{'32' if flag else '16'}-channel blocks, rows {tyw or 'default'}"
        assert np.array_equal(hv.view(np.uint32), outs[0][0].view(np.uint32)), name
        assert bv == outs[0][1], name
    log(f"H={H} W={W} w={w} h={h} g={g} k={k}: {len(CHOICES)} tile choices agree, max err {err.max():.3e}")


@pytest.mark.parametrize("tuned", [False, True])
def test_batched_equals_single_pair(tuned):
    """tuned=False: autotuning off, the batch's default 16-channel blocks;
    True: the first call's result comes from the tuner's last candidate,
    32-channel blocks at 256 rows."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = B.Context(stream=torch.cuda.current_stream())
    B.vqnnf_ctx_set_autotune(ctx, 1 if tuned else 0)
    # templates of grid 2 and 3, equal and unequal bins, k from 16 to 64
    wl = synth.make_multi_template(77, 176, 208, 64, 32, 0.3, "bf16", 6, (14, 60), (16, 32, 64), 2)
    wl3 = synth.make_multi_template(78, 176, 208, 64, 32, 0.3, "bf16", 4, (14, 60), (32, 64), 3)
    maps = wl.maps + wl3.maps
    devs = [torch.from_numpy(qm.data.view(np.int16)).cuda() for qm in maps]
    tpls, fms, heats = [], [], []
    for mi, row in enumerate(wl.templates + wl3.templates):
        for t in row:
            hh, ww, _ = t.data.shape
            tpls.append(B.vqnnf_codebook(ctx, t.data, t.k, 10, 0, B.default_bank(ww, hh, t.grid)))
            fms.append(B.device_fmap(devs[mi], "bf16"))
            heats.append(torch.full(((maps[mi].H - hh + 1) * (maps[mi].W - ww + 1),), float("nan"),
                                    device="cuda"))
    P = B.VQNNF_PREC_BF16_REFINED
    out = B.vqnnf_match_batched(ctx, tpls, fms, P, heats)
    for i, (tp, fm, ht) in enumerate(zip(tpls, fms, heats)):
        ref = torch.empty_like(ht)
        best = B.vqnnf_match(ctx, tp, fm, P, ref)
        assert torch.equal(ht, ref), f"pair {i}"
        assert out[i] == best, f"pair {i}"
    log(f"tuned={tuned}: {len(tpls)} batched pairs equal the single-pair path")
    torch.cuda.synchronize()
    for tp in tpls:
        tp.free()
    ctx.close()
