"""C-ABI checks that need no GPU: the library loads and exports every symbol
include/vqnnf.h declares; a host-only context prepares templates whose
codebook, NNF and counts equal the oracle's bit for bit; argument errors and
the scratch cap are reported before any HIP call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import vqnnf_oracle as O
from paper_2306_15010_amd import binding as B
from paper_2306_15010_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "vqnnf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vqnnf_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = B.lib()
    names = _header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(B.EXPORTED)
    assert B.vqnnf_version().startswith("vqnnf-gfx950")


def _oracle_codebook(t, k, iters, seed):
    return O.kmeans_codebook(t, k, iters, seed)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_host_kmeans_matches_oracle_bit_for_bit(seed):
    ctx = B.Context(host=True)
    wl = synth.make_config("c1", seed=synth.MASTER_SEED + 17 * seed)
    t = wl.templates[0][0]
    tpl = B.vqnnf_codebook(ctx, t.data, t.k, 20, seed, B.default_bank(16, 16, t.grid))
    cb = tpl.codebook()
    ref = _oracle_codebook(t.data, t.k, 20, seed)
    assert np.array_equal(cb.view(np.uint32), ref.view(np.uint32))
    tl = O.assign_map(t.data.astype(np.float64), ref.astype(np.float64))
    assert np.array_equal(tpl.labels(), tl.astype(np.uint8))
    filters = O.expand_bank(O.default_bank(16, 16, t.grid))
    rt = O.template_representation(tl, t.k, filters)
    assert np.array_equal(tpl.counts(), rt.astype(np.int32))
    np.testing.assert_array_equal(tpl.weights(), np.array([f.weight for f in filters], np.float32))


def test_host_kmeans_matches_oracle_larger():
    # 48x48 template, D=64, k=32 (the 512x512 benchmark's template shape)
    rng = np.random.default_rng(4)
    qm = synth.random_map(48, 48, 64, "f32", seed=5, M=40)
    ctx = B.Context(host=True)
    tpl = B.vqnnf_codebook(ctx, qm.data, 32, 20, 7, B.default_bank(48, 48, 3))
    ref = O.kmeans_codebook(qm.data, 32, 20, 7)
    assert np.array_equal(tpl.codebook().view(np.uint32), ref.view(np.uint32))


def test_template_from_codebook_round_trip():
    ctx = B.Context(host=True)
    qm = synth.random_map(12, 10, 9, "f32", seed=3, M=6)
    cb = O.kmeans_codebook(qm.data, 5, 10, 1)
    tpl = B.vqnnf_template_from_codebook(ctx, qm.data, cb, [(0, 0, 10, 12, 1, 1, 1.0)])
    assert np.array_equal(tpl.codebook(), cb)
    assert np.array_equal(tpl.labels(), O.assign_map(qm.data.astype(np.float64),
                                                     cb.astype(np.float64)).astype(np.uint8))


def _status_of(fn):
    with pytest.raises(B.VqnnfError) as ei:
        fn()
    return ei.value.status


def test_argument_errors_on_host_context():
    ctx = B.Context(host=True)
    t = np.zeros((8, 8, 4), np.float32)
    t[..., 0] = np.arange(64).reshape(8, 8)
    bank = B.default_bank(8, 8, 2)
    assert _status_of(lambda: B.vqnnf_codebook(ctx, t, 0, 5, 0, bank)) == B.VQNNF_EINVAL
    assert _status_of(lambda: B.vqnnf_codebook(ctx, t, 257, 5, 0, bank)) == B.VQNNF_EINVAL
    assert _status_of(lambda: B.vqnnf_codebook(ctx, t, 4, -1, 0, bank)) == B.VQNNF_EINVAL
    assert _status_of(lambda: B.vqnnf_codebook(ctx, t, 4, 5, 0, [(0, 0, 9, 8, 1, 1, 1.0)])) == B.VQNNF_EINVAL
    assert _status_of(lambda: B.vqnnf_codebook(ctx, t, 4, 5, 0, [(0, 0, 8, 8, 9, 1, 1.0)])) == B.VQNNF_EINVAL
    bad = t.copy()
    bad[2, 3, 1] = np.nan
    assert _status_of(lambda: B.vqnnf_codebook(ctx, bad, 4, 5, 0, bank)) == B.VQNNF_EINVAL
    tpl = B.vqnnf_codebook(ctx, t, 4, 5, 0, bank)
    L = B.lib()

    class FakeTensor:
        def __init__(self, p):
            self.p = p

        def data_ptr(self):
            return self.p

    q = B.FMap(0x1000, B.VQNNF_BF16, 32, 32, 4, 4, None)
    lab = FakeTensor(0x2000)
    # the query pointer is never dereferenced on a host context
    with pytest.raises(B.VqnnfError) as ei:
        B.vqnnf_assign(ctx, tpl, q, B.VQNNF_PREC_BF16_REFINED, lab)
    assert ei.value.status == B.VQNNF_ENOTSUP
    q_bad_d = B.FMap(0x1000, B.VQNNF_BF16, 32, 32, 5, 5, None)
    assert _status_of(lambda: B.vqnnf_assign(ctx, tpl, q_bad_d, 1, lab)) == B.VQNNF_EINVAL
    q_bad_dt = B.FMap(0x1000, 7, 32, 32, 4, 4, None)
    assert _status_of(lambda: B.vqnnf_assign(ctx, tpl, q_bad_dt, 1, lab)) == B.VQNNF_EINVAL
    q_stride = B.FMap(0x1000, B.VQNNF_BF16, 32, 32, 4, 3, None)
    assert _status_of(lambda: B.vqnnf_assign(ctx, tpl, q_stride, 1, lab)) == B.VQNNF_EINVAL
    assert _status_of(lambda: B.vqnnf_assign(ctx, tpl, q, 9, lab)) == B.VQNNF_EINVAL
    # the FP8 precision is for FP8 maps only
    assert _status_of(lambda: B.vqnnf_assign(ctx, tpl, q, B.VQNNF_PREC_FP8_REFINED, lab)) == B.VQNNF_EINVAL
    assert "FP8" in B.last_error()
    sc8 = np.ones(4, np.float32)
    q8ok = B.FMap(0x1000, B.VQNNF_FP8_E4M3, 32, 32, 4, 4, sc8.ctypes.data)
    assert _status_of(lambda: B.vqnnf_assign(ctx, tpl, q8ok, B.VQNNF_PREC_FP8_REFINED, lab)) == B.VQNNF_ENOTSUP
    q_null = B.FMap(None, B.VQNNF_BF16, 32, 32, 4, 4, None)
    assert _status_of(lambda: B.vqnnf_assign(ctx, tpl, q_null, 1, lab)) == B.VQNNF_EINVAL
    # empty maps and maps at the size cap (H*W < 2^31, so 32-bit pixel
    # indices and worklist offsets cannot wrap) are rejected before any device call
    for Hh, Ww in ((0, 32), (32, 0), (65536, 32768)):
        q_e = B.FMap(0x1000, B.VQNNF_BF16, Hh, Ww, 4, 4, None)
        assert _status_of(lambda: B.vqnnf_assign(ctx, tpl, q_e, 1, lab)) == B.VQNNF_EINVAL
        assert _status_of(lambda: B.vqnnf_match(ctx, tpl, q_e, 1, FakeTensor(0x3000))) == B.VQNNF_EINVAL
    assert "2^31" in B.last_error()
    assert _status_of(lambda: B.vqnnf_score(ctx, tpl, lab, 0, 32, FakeTensor(0x3000))) == B.VQNNF_EINVAL
    assert _status_of(lambda: B.vqnnf_score(ctx, tpl, lab, 65536, 32768, FakeTensor(0x3000))) == B.VQNNF_EINVAL
    # template larger than the map
    q_small = B.FMap(0x1000, B.VQNNF_BF16, 7, 32, 4, 4, None)
    assert _status_of(lambda: B.vqnnf_match(ctx, tpl, q_small, 1, FakeTensor(0x3000))) == B.VQNNF_EINVAL
    assert _status_of(lambda: B.vqnnf_score(ctx, tpl, lab, 32, 7, FakeTensor(0x3000))) == B.VQNNF_EINVAL
    # FP8 maps: the host channel scales must be present, finite and >= 0
    sc = np.ones(4, np.float32)
    q8 = B.FMap(0x1000, B.VQNNF_FP8_E4M3, 32, 32, 4, 4, None)
    assert _status_of(lambda: B.vqnnf_assign(ctx, tpl, q8, 1, lab)) == B.VQNNF_EINVAL
    for bad_s in (np.float32(-1.0), np.float32(np.nan), np.float32(np.inf)):
        sc_bad = sc.copy()
        sc_bad[2] = bad_s
        q8b = B.FMap(0x1000, B.VQNNF_FP8_E4M3, 32, 32, 4, 4, sc_bad.ctypes.data)
        assert _status_of(lambda: B.vqnnf_assign(ctx, tpl, q8b, 1, lab)) == B.VQNNF_EINVAL
    q8ok = B.FMap(0x1000, B.VQNNF_FP8_E4M3, 32, 32, 4, 4, sc.ctypes.data)
    assert _status_of(lambda: B.vqnnf_assign(ctx, tpl, q8ok, 1, lab)) == B.VQNNF_ENOTSUP
    # batched: every pair is validated before anything runs; errors name the pair
    with pytest.raises(B.VqnnfError) as ei:
        B.vqnnf_match_batched(ctx, [tpl, tpl], [q, q_bad_d], 1, [FakeTensor(0x3000)] * 2)
    assert ei.value.status == B.VQNNF_EINVAL and "pair 1" in str(ei.value)
    with pytest.raises(B.VqnnfError) as ei:
        B.vqnnf_match_batched(ctx, [tpl], [q_small], 1, [FakeTensor(0x3000)])
    assert ei.value.status == B.VQNNF_EINVAL and "pair 0" in str(ei.value)
    assert L.vqnnf_match_batched(ctx.h, 0, None, None, 1, None, None, None) == B.VQNNF_EINVAL
    with pytest.raises(B.VqnnfError) as ei:   # valid pairs: needs a device
        B.vqnnf_match_batched(ctx, [tpl, tpl], [q, q], 1, [FakeTensor(0x3000)] * 2)
    assert ei.value.status == B.VQNNF_ENOTSUP
    assert L.vqnnf_ctx_set_graph(ctx.h, 1) == B.VQNNF_ENOTSUP
    # freed handles
    tpl.free()
    h = C.c_void_p(0)
    st = L.vqnnf_template_info(h, None, None, None, None, None)
    assert st == B.VQNNF_EHANDLE


def test_scratch_cap_reports_enomem_before_any_device_call():
    ctx = B.Context(host=True, scratch_cap=1 << 18)
    t = np.random.default_rng(0).standard_normal((8, 8, 4)).astype(np.float32)
    tpl = B.vqnnf_codebook(ctx, t, 4, 5, 0, B.default_bank(8, 8, 2))

    class FakeTensor:
        def data_ptr(self):
            return 0x2000

    q = B.FMap(0x1000, B.VQNNF_BF16, 1024, 1024, 4, 4, None)
    with pytest.raises(B.VqnnfError) as ei:
        B.vqnnf_assign(ctx, tpl, q, B.VQNNF_PREC_BF16_REFINED, FakeTensor())
    assert ei.value.status == B.VQNNF_ENOMEM
    with pytest.raises(B.VqnnfError) as ei:
        B.vqnnf_filter(ctx, tpl, FakeTensor(), 1024, 1024, FakeTensor())
    assert ei.value.status == B.VQNNF_ENOMEM


def test_batched_codebooks_on_host_context():
    ctx = B.Context(host=True)
    ts = [synth.random_map(h, w, 12, "f32", seed=60 + h, M=8).data for h, w in [(10, 12), (14, 9), (8, 8)]]
    ks, seeds = [4, 8, 5], [1, 2, 3]
    banks = [B.default_bank(12, 10, 2), B.paper_bank(9, 14, "3rect", 1), B.default_bank(8, 8, 1)]
    out = B.vqnnf_codebook_batched(ctx, ts, ks, 20, seeds, banks)
    for i, tp in enumerate(out):
        one = B.vqnnf_codebook(ctx, ts[i], ks[i], 20, seeds[i], banks[i])
        assert np.array_equal(tp.codebook().view(np.uint32), one.codebook().view(np.uint32))
        assert np.array_equal(tp.labels(), one.labels())
        assert np.array_equal(tp.responses(), one.responses())
    with pytest.raises(B.VqnnfError) as ei:
        B.vqnnf_codebook_batched(ctx, ts, [4, 0, 5], 20, seeds, banks)
    assert ei.value.status == B.VQNNF_EINVAL and "template 1" in str(ei.value)


def test_large_template_non_finite_names_first_pixel():
    """A large template is scanned for non-finite values on several threads;
    the error still names the first such pixel in row-major order."""
    ctx = B.Context(host=True)
    t = np.ones((255, 255, 80), np.float32)
    t[200, 17, 3] = np.inf
    t[120, 250, 79] = np.nan
    t[254, 254, 0] = -np.inf
    assert _status_of(lambda: B.vqnnf_codebook(ctx, t, 4, 1, 0, B.default_bank(255, 255, 1))) == B.VQNNF_EINVAL
    assert f"pixel {120 * 255 + 250}" in B.last_error(), B.last_error()
    t[120, 250, 79] = 1.0
    t[200, 17, 3] = 1.0
    assert _status_of(lambda: B.vqnnf_codebook(ctx, t, 4, 1, 0, B.default_bank(255, 255, 1))) == B.VQNNF_EINVAL
    assert f"pixel {254 * 255 + 254}" in B.last_error(), B.last_error()
