"""vqnnf_match_noalloc (the matching call that allocates nothing) against
vqnnf_match, through the C ABI: two calls in a row on each path, the second
with a smaller map (the fixed array keeps the first call's contents), for
the refined and plain paths and BF16 / FP32 / FP8 storage.  Heatmaps and best
windows must be identical bit for bit; the size limit and the FP8 table
precondition must be reported as errors."""
import sys

import numpy as np
import pytest

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


def _pair(ctx, qm, tpl, prec):
    h, w = tpl.height, tpl.w
    n = (qm.H - h + 1) * (qm.W - w + 1)
    dq = _dev(qm)
    fm = B.device_fmap(dq, qm.dtype, qm.scale)
    ref = torch.full((n,), float("nan"), device="cuda")
    got = torch.full((n,), float("nan"), device="cuda")
    best_ref = B.vqnnf_match(ctx, tpl, fm, prec, ref)
    return dq, fm, ref, got, best_ref


@pytest.mark.parametrize("dtype,prec", [("bf16", B.VQNNF_PREC_BF16_REFINED),
                                        ("bf16", B.VQNNF_PREC_FP32_PLAIN),
                                        ("f32", B.VQNNF_PREC_BF16_REFINED),
                                        ("fp8", B.VQNNF_PREC_FP8_REFINED)])
def test_noalloc_matches_vqnnf_match(dtype, prec):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = B.Context(stream=torch.cuda.current_stream())
    D, k, side = 64, 32, 24
    big = synth.random_map(200, 232, D, dtype, seed=7101)
    small = synth.random_map(77, 91, D, dtype, seed=7102)
    rng = np.random.default_rng(7103)
    tmpl = np.ascontiguousarray(synth.bf16_bits_to_f32(synth.f32_to_bf16_bits(
        rng.standard_normal((side, side, D)).astype(np.float32))))
    tpl = B.vqnnf_codebook(ctx, tmpl, k, 20, 3, B.default_bank(side, side, 3))
    for qm in (big, small):     # the second call has the smaller input
        log(f"{dtype} prec {prec}: {qm.W}x{qm.H} map")
        dq, fm, ref, got, best_ref = _pair(ctx, qm, tpl, prec)
        best = B.vqnnf_match_noalloc(ctx, tpl, fm, prec, got)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), "heatmap differs from vqnnf_match"
        assert best == best_ref, (best, best_ref)
        # without the host outputs (no synchronisation inside the call)
        got.fill_(float("nan"))
        assert B.vqnnf_match_noalloc(ctx, tpl, fm, prec, got, want_best=False) is None
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
    ctx.close()


def test_noalloc_full_size_workload_and_limits():
    """The 1024x1024 D=512 BF16 k=128 pair fits the fixed array; a map that
    does not fit is refused with ENOMEM, and an FP8 map whose scales have no
    tables yet with EINVAL."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = B.Context(stream=torch.cuda.current_stream())
    D, k, side = 512, 128, 96
    rng = np.random.default_rng(7104)
    tmpl = rng.standard_normal((side, side, D)).astype(np.float32)
    tpl = B.vqnnf_codebook(ctx, tmpl, k, 2, 5, B.default_bank(side, side, 3))
    for (H, W) in ((1024, 1024), (300, 517)):
        log(f"noalloc refined {W}x{H} D=512 k=128")
        q = torch.from_numpy(synth.f32_to_bf16_bits(
            rng.standard_normal((H, W, D)).astype(np.float32)).view(np.int16)).cuda()
        fm = B.device_fmap(q, "bf16")
        n = (H - side + 1) * (W - side + 1)
        ref = torch.empty(n, device="cuda")
        got = torch.empty(n, device="cuda")
        best_ref = B.vqnnf_match(ctx, tpl, fm, B.VQNNF_PREC_BF16_REFINED, ref)
        best = B.vqnnf_match_noalloc(ctx, tpl, fm, B.VQNNF_PREC_BF16_REFINED, got)
        torch.cuda.synchronize()
        assert torch.equal(got, ref) and best == best_ref
        del q, ref, got
    # too large for the array: refused before anything is enqueued
    H, W = 2048, 2048
    q = torch.zeros((H, W, D), dtype=torch.int16, device="cuda")
    heat = torch.empty((H - side + 1) * (W - side + 1), device="cuda")
    with pytest.raises(B.VqnnfError) as ei:
        B.vqnnf_match_noalloc(ctx, tpl, B.device_fmap(q, "bf16"), B.VQNNF_PREC_BF16_REFINED, heat)
    assert ei.value.status == B.VQNNF_ENOMEM
    del q, heat
    # FP8 map with scales the template has no tables for
    small = synth.random_map(64, 64, D, "fp8", seed=7105)
    dq = _dev(small)
    tpl8 = B.vqnnf_codebook(ctx, tmpl[:32, :32], 16, 2, 6, B.default_bank(32, 32, 2))
    heat = torch.empty((64 - 31) * (64 - 31), device="cuda")
    with pytest.raises(B.VqnnfError) as ei:
        B.vqnnf_match_noalloc(ctx, tpl8, B.device_fmap(dq, "fp8", small.scale),
                              B.VQNNF_PREC_FP8_REFINED, heat)
    assert ei.value.status == B.VQNNF_EINVAL
    ctx.close()
