"""Weighted filter banks through the C ABI on a host-only context (no GPU):
the library's version of the paper's bank (vqnnf_paper_bank) against the
oracle's independent one, the template representation R(tau) of weighted and
mixed banks against the FP64 oracle, and the argument errors."""
import ctypes as C

import numpy as np
import pytest

from oracle import vqnnf_oracle as O
from paper_2306_15010_amd import binding as B
from paper_2306_15010_amd import synth

U = 2.0 ** -24


def _status_of(fn):
    with pytest.raises(B.VqnnfError) as ei:
        fn()
    return ei.value.status


@pytest.mark.parametrize("w,h,fs,S", [(96, 96, "23rect", 3), (100, 60, "23rect", 4), (37, 41, "2rect", 2),
                                      (9, 12, "3rect", 3), (40, 40, "gauss", 1)])
def test_library_bank_equals_oracle_bank(w, h, fs, S):
    lib_bank = B.paper_bank(w, h, fs, S)
    ora_bank = O.paper_bank(w, h, fs, S)
    assert len(lib_bank) == len(ora_bank)
    for (x0, y0, x1, y1, gx, gy, wt, bw), d in zip(lib_bank, ora_bank):
        assert (x0, y0, x1, y1, gx, gy) == (d.x0, d.y0, d.x1, d.y1, d.gx, d.gy)
        assert wt == np.float32(d.weight)
        # FP32 coefficients: the oracle's FP64 values rounded once
        np.testing.assert_allclose(bw, d.bin_weight, rtol=U, atol=0)


def test_paper_bank_errors():
    assert _status_of(lambda: B.paper_bank(40, 40, 7, 2)) == B.VQNNF_EINVAL
    assert _status_of(lambda: B.paper_bank(40, 40, "gauss", 0)) == B.VQNNF_EINVAL
    assert _status_of(lambda: B.paper_bank(8, 8, "gauss", 3)) == B.VQNNF_EINVAL   # 2x2 sub-window
    arr = (B.FilterDesc * 4)()
    bw = np.zeros(36, np.float32)
    n = C.c_int32(-1)
    st = B.lib().vqnnf_paper_bank(40, 40, B.VQNNF_BANK_23RECT, 1, arr, bw.ctypes.data, 4, C.byref(n))
    assert st == B.VQNNF_EINVAL and n.value == -1        # 5 descs do not fit in 4


def _template(seed, h, w, D=6, M=10):
    return synth.random_map(h, w, D, "f32", seed=seed, M=M).data


def _oracle_rt(tpl, data, bank_o, seed):
    """R(tau) by the oracle from its own k-means (20 iterations, `seed`); the
    library's codebook and template labels must equal the oracle's."""
    cb32 = O.kmeans_codebook(data, tpl.k, 20, seed)
    assert np.array_equal(tpl.codebook().view(np.uint32), cb32.view(np.uint32))
    tl = O.assign_map(data.astype(np.float64), cb32.astype(np.float64))
    assert np.array_equal(tpl.labels().astype(np.int64), tl)
    return O.template_representation(tl, tpl.k, O.expand_bank(bank_o))


def _to_oracle(bank):
    out = []
    for e in bank:
        x0, y0, x1, y1, gx, gy, wt = e[:7]
        bw = None if len(e) < 8 or e[7] is None else np.asarray(e[7], np.float64)
        out.append(O.FilterDesc(x0, y0, x1, y1, gx, gy, bw, float(wt)))
    return out


def _resp_bound(bank_o, k):
    """|R_lib - R_oracle| per filter: FP32 coefficients (one rounding each)
    and an FMA chain over at most 16 bins: (nb + 1) * u * sum_b |coef_b| * n_b;
    sum over one channel of |coef| * n is at most max|coef| * area(region)."""
    out = []
    for f in O.expand_bank(bank_o):
        nb = len(f.boxes)
        mx = max(abs(c) for c, *_ in f.boxes)
        area = sum((x1 - x0) * (y1 - y0) for _, x0, y0, x1, y1 in f.boxes)
        out.append((nb + 1) * U * mx * area)
    return np.array(out)[:, None]


@pytest.mark.parametrize("fs,S", [("23rect", 3), ("2rect", 2), ("gauss", 1)])
def test_weighted_template_responses_match_oracle(fs, S):
    ctx = B.Context(host=True)
    h, w, k = 36, 30, 12
    data = _template(21, h, w)
    bank = B.paper_bank(w, h, fs, S)
    tpl = B.vqnnf_codebook(ctx, data, k, 20, 3, bank)
    bank_o = _to_oracle(bank)           # the library's FP32 coefficients, read exactly
    rt = _oracle_rt(tpl, data, bank_o, 3)
    r = tpl.responses().astype(np.float64)
    assert r.shape == rt.shape == (len(bank), k)
    assert np.all(np.abs(r - rt) <= _resp_bound(bank_o, k))
    np.testing.assert_array_equal(tpl.weights(), np.array([e[6] for e in bank], np.float32))
    assert _status_of(lambda: tpl.counts()) == B.VQNNF_ENOTSUP


def test_mixed_bank_responses():
    """Indicator entries (a 2x2 grid and a 5x5 grid, larger than a weighted
    group may be) next to a weighted one: indicator responses are exact counts."""
    ctx = B.Context(host=True)
    h, w, k = 25, 27, 9
    data = _template(22, h, w)
    rng = np.random.default_rng(5)
    bank = [(0, 0, w, h, 1, 1, 1.0), (2, 3, 22, 21, 2, 2, 0.5), (0, 0, w, h, 5, 5, 1.0),
            (4, 1, 20, 24, 4, 3, 0.3, rng.standard_normal((3, 4)))]
    tpl = B.vqnnf_codebook(ctx, data, k, 20, 4, bank)
    bank_o = _to_oracle(bank)
    rt = _oracle_rt(tpl, data, bank_o, 4)
    r = tpl.responses().astype(np.float64)
    assert r.shape == (1 + 4 + 25 + 1, k)
    assert np.array_equal(r[:30], rt[:30])
    assert np.all(np.abs(r[30] - rt[30]) <= _resp_bound(bank_o, k)[30])
    wo = np.array([f.weight for f in O.expand_bank(bank_o)], np.float32)
    np.testing.assert_array_equal(tpl.weights(), wo)


def test_indicator_bank_responses_are_counts():
    ctx = B.Context(host=True)
    tpl = B.vqnnf_codebook(ctx, _template(23, 16, 16), 8, 20, 0, B.default_bank(16, 16, 3))
    assert np.array_equal(tpl.responses(), tpl.counts().astype(np.float32))


def test_weighted_bank_errors():
    ctx = B.Context(host=True)
    t = _template(24, 20, 20)
    big = (0, 0, 20, 20, 5, 4, 1.0, np.ones((4, 5)))
    assert _status_of(lambda: B.vqnnf_codebook(ctx, t, 4, 5, 0, [big])) == B.VQNNF_ENOTSUP
    nanw = np.ones((3, 3))
    nanw[1, 2] = np.nan
    assert _status_of(lambda: B.vqnnf_codebook(ctx, t, 4, 5, 0, [(0, 0, 20, 20, 3, 3, 1.0, nanw)])) \
        == B.VQNNF_EINVAL
    assert _status_of(lambda: B.vqnnf_codebook(ctx, t, 4, 5, 0, [(0, 0, 21, 20, 3, 3, 1.0, np.ones((3, 3)))])) \
        == B.VQNNF_EINVAL
    # the on-chip score takes only the full-window + grid indicator bank
    tpl = B.vqnnf_codebook(ctx, t, 4, 5, 0, B.paper_bank(20, 20, "2rect", 2))

    class FakeTensor:
        def __init__(self, p):
            self.p = p

        def data_ptr(self):
            return self.p

    with pytest.raises(B.VqnnfError) as ei:
        B.vqnnf_score(ctx, tpl, FakeTensor(0x2000), 32, 32, FakeTensor(0x3000))
    assert ei.value.status == B.VQNNF_ENOTSUP and "vqnnf_score_integral" in str(ei.value)


def test_rgb_template_on_host_context_matches_oracle():
    """An RGB template: its colour features (3x3 patches), k-means codebook and
    NNF equal the oracle's bit for bit."""
    ctx = B.Context(host=True)
    img = synth.rgb_image(30, 34, seed=5)
    tpl = B.vqnnf_codebook(ctx, img, 12, 20, 2, B.default_bank(34, 30, 2))
    feats = O.rgb_patch_features(img)
    ref = O.kmeans_codebook(feats.astype(np.float32), 12, 20, 2)
    assert np.array_equal(tpl.codebook().view(np.uint32), ref.view(np.uint32))
    assert np.array_equal(tpl.labels(), O.assign_map(feats, ref.astype(np.float64)).astype(np.uint8))
    # an RGB map must declare its 27 colour features
    bad = B.FMap(img.ctypes.data, B.VQNNF_RGB8, 30, 34, 26, 3, None)
    h = C.c_void_p()
    st = B.lib().vqnnf_codebook(ctx.h, C.byref(bad), 4, 5, 0, B.bank_descs(B.default_bank(34, 30, 2)), 2,
                                C.byref(h))
    assert st == B.VQNNF_EINVAL
