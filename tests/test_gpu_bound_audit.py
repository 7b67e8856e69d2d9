"""Audit of the refined search's error bound on the real kernel.

The labels of the refined path are exact only if the FP32 scores the
matrix-core kernel produces, s~_j = ||c_j||^2 - 2 q.c_j, never differ from
the exact s_j by more than the per-codeword bound A0 + A1 * ||q|| that the
flag threshold is built from.  Here the kernel writes every (pixel,
codeword) score (vqnnf_ctx_set_debug_scores) and each one is checked against
the exact value, computed in FP64 from the decoded inputs (every product of a
stored element and an FP32 codeword value is exact in FP64; the FP64 sum's
own rounding, at most (D + 2) 2^-52 (||c||^2 + 2 sum |q||c|), is allowed on
top).  Inputs: random smooth maps, a large query norm, exact dyadic tie
midpoints with duplicated codewords, k = 256 at D = 512, FP32, BF16 and FP8
storage, and a D that is not a multiple of 64 (the bounds-checked load path).
The largest observed error / bound ratio of every case is printed."""
import sys
import zlib

import numpy as np
import pytest

from oracle import vqnnf_oracle as O
from paper_2306_15010_amd import binding as B
from paper_2306_15010_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _dev(qm):
    if qm.dtype == "bf16":
        return torch.from_numpy(qm.data.view(np.int16)).cuda()
    return torch.from_numpy(np.ascontiguousarray(qm.data)).cuda()


def _case_maps(name):
    """(query map, codebook FP32 [k, D]) of a case."""
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    if name == "tie_midpoints":
        D, k = 64, 32
        cb = (rng.integers(-32, 33, size=(k, D)) / 8.0).astype(np.float32)
        cb[5] = cb[4]                      # duplicated codewords
        cb[17] = cb[4]
        a, b = rng.integers(0, k, size=(2, 48 * 40))
        q = ((cb[a].astype(np.float64) + cb[b]) / 2.0).reshape(48, 40, D).astype(np.float32)
        return synth.encode(q, "bf16"), cb
    spec = {"bf16_d512_k256": ("bf16", 512, 256, 1.0), "bf16_d512_k128_large_norm": ("bf16", 512, 128, 1024.0),
            "f32_d64_k32": ("f32", 64, 32, 1.0), "fp8_d256_k64": ("fp8", 256, 64, 1.0),
            "bf16_d40_k12": ("bf16", 40, 12, 1.0), "f32_d96_k48_large_norm": ("f32", 96, 48, 3.0e3)}[name]
    dtype, D, k, scale = spec
    q = synth.random_map(48, 40, D, "f32", seed=int(rng.integers(0, 2 ** 31)), M=8).data * np.float32(scale)
    qm = synth.encode(np.ascontiguousarray(q, dtype=np.float32), dtype)
    src = O.decode(dtype, qm.data, qm.scale).reshape(-1, D)
    cb = (src[rng.integers(0, len(src), size=k)] + 0.02 * scale * rng.standard_normal((k, D))).astype(np.float32)
    return qm, cb


CASES = ["bf16_d512_k256", "bf16_d512_k128_large_norm", "tie_midpoints", "f32_d64_k32", "fp8_d256_k64",
         "bf16_d40_k12", "f32_d96_k48_large_norm"]


@pytest.mark.parametrize("name", CASES)
def test_refined_scores_within_bound(name):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qm, cb = _case_maps(name)
    k, D = cb.shape
    ctx = B.Context(stream=torch.cuda.current_stream())
    side = 8
    tmpl = np.ascontiguousarray(O.decode(qm.dtype, qm.data[:side, :side], qm.scale).astype(np.float32))
    tpl = B.vqnnf_template_from_codebook(ctx, tmpl, cb, B.default_bank(side, side, 2))
    kpad = (k + 15) // 16 * 16
    n = qm.H * qm.W
    scores = torch.full((n * kpad,), float("nan"), device="cuda")
    B.vqnnf_ctx_set_debug_scores(ctx, scores)
    lab = torch.empty(n, dtype=torch.uint8, device="cuda")
    dq = _dev(qm)
    B.vqnnf_assign(ctx, tpl, B.device_fmap(dq, qm.dtype, qm.scale), B.VQNNF_PREC_BF16_REFINED, lab)
    B.vqnnf_ctx_set_debug_scores(ctx, None)
    torch.cuda.synchronize()
    st = scores.cpu().numpy().reshape(n, kpad)[:, :k].astype(np.float64)
    assert np.isfinite(st).all()
    a0, a1, a2, A0, A1 = B.vqnnf_template_score_bound(tpl, qm.dtype, qm.scale)
    q = O.decode(qm.dtype, qm.data, qm.scale).reshape(n, D)
    c = cb.astype(np.float64)
    cn2 = np.einsum("jd,jd->j", c, c)
    exact = cn2[None, :] - 2.0 * (q @ c.T)
    slack = (D + 2) * 2.0 ** -52 * (cn2[None, :] + 2.0 * (np.abs(q) @ np.abs(c).T))
    # the bound's norm is that of the stored values (FP8: the E4M3 code values)
    stored = q if qm.dtype != "fp8" else O.decode("fp8", qm.data, np.ones(D, np.float32)).reshape(n, D)
    nq = np.sqrt(np.einsum("pd,pd->p", stored, stored))
    bound = A0 + A1 * nq
    err = np.abs(st - exact)
    ratio = err / bound[:, None]
    log(f"{name}: max |s~ - s| = {err.max():.3e}, max error / bound = {ratio.max():.4f} "
        f"(A0 {A0:.3e}, A1 {A1:.3e}, ||q|| up to {nq.max():.3e})")
    assert np.all(err <= bound[:, None] + slack), f"{int((err > bound[:, None] + slack).sum())} scores outside"
    # the threshold the kernel applies covers the bound twice plus the FP64 term
    thr = a0 + nq * (a1 + nq * a2)
    assert np.all(thr >= 2 * bound)
    # and the labels are still the oracle's
    assert np.array_equal(lab.cpu().numpy().astype(np.int64), O.assign(q, c))
    ctx.close()
