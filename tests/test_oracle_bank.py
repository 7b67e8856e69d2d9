"""Pins for the oracle's version of the paper's filter bank (O5b): Gaussian and
Haar-like coarse filters on a 3x3 grid, sub-scale aggregation and the scale
weights (Sec. 3.2.2, Sec. 3.3 eq. 2, Sec. 5.2 "Filtering"; Supp. S.3 option c).

The filter counts the paper states for its best banks pin the composition; closed
forms on hand-built label maps pin the orientation and sign of each filter; mirror
and transpose symmetries pin the geometry against x/y or left/right mix-ups."""
import math

import numpy as np
import pytest

from oracle import vqnnf_oracle as O


def test_filter_counts_stated_in_the_paper():
    # Sec. 5.2: F_2-rect at S = 3 is 9 filters, F_2,3-rect at S = 3 is 15 and at S = 4 is 20
    assert len(O.paper_bank(96, 96, "2rect", 3)) == 9
    assert len(O.paper_bank(96, 96, "23rect", 3)) == 15
    assert len(O.paper_bank(100, 100, "23rect", 4)) == 20
    assert len(O.paper_bank(40, 40, "gauss", 1)) == 1
    # the Haar sets also hold the Gaussian
    for fs in ("2rect", "3rect", "23rect"):
        bank = O.paper_bank(48, 48, fs, 2)
        assert sum(np.array_equal(d.bin_weight, O.gaussian_coarse()) for d in bank) == 2


def test_gaussian_closed_form():
    g = O.gaussian_coarse()
    assert g[1, 1] == 1.0
    for b, a in [(0, 1), (1, 0), (1, 2), (2, 1)]:
        assert g[b, a] == pytest.approx(math.exp(-1.0 / 8.0), rel=1e-15)
    for b, a in [(0, 0), (0, 2), (2, 0), (2, 2)]:
        assert g[b, a] == pytest.approx(math.exp(-1.0 / 4.0), rel=1e-15)
    assert np.array_equal(g, g.T) and np.array_equal(g, g[::-1, ::-1])


def test_haar_shapes():
    g = O.gaussian_coarse()
    h2x, h3x = O.coarse_filter("haar2x"), O.coarse_filter("haar3x")
    assert np.array_equal(h2x[:, 0], g[:, 0]) and np.all(h2x[:, 1] == 0) and np.array_equal(h2x[:, 2], -g[:, 2])
    assert np.array_equal(h3x[:, 0], g[:, 0]) and np.array_equal(h3x[:, 1], -2 * g[:, 1])
    assert np.array_equal(h3x[:, 2], g[:, 2])
    assert np.array_equal(O.coarse_filter("haar2y"), h2x.T)
    assert np.array_equal(O.coarse_filter("haar3y"), h3x.T)


def test_subscale_regions_and_weights():
    # hand-computed centred sub-windows of a 100 x 60 template
    assert O.subscale_region(100, 60, 1) == (0, 0, 100, 60)
    assert O.subscale_region(100, 60, 2) == (25, 15, 75, 45)
    assert O.subscale_region(100, 60, 3) == (33, 20, 66, 40)
    assert O.subscale_region(100, 60, 4) == (37, 22, 62, 37)
    bank = O.paper_bank(100, 60, "23rect", 4)
    for i, d in enumerate(bank):
        s, f = 1 + i // 5, i % 5
        assert (d.x0, d.y0, d.x1, d.y1) == O.subscale_region(100, 60, s)
        assert (d.gx, d.gy) == (3, 3)
        assert d.weight == (1.0 if f == 0 else 0.25) / s
    with pytest.raises(ValueError):
        O.paper_bank(8, 8, "gauss", 3)           # 2 x 2 sub-window: empty bins


def test_responses_on_a_left_third_split():
    """Region 36 x 36, bins 12 x 12; label 0 in the left column of bins, label 1
    elsewhere.  Each bin holds 1/9 of the region, so a filter's response on
    channel j is (1/9) * sum of its weights over the bins labelled j."""
    lab = np.ones((36, 36), dtype=np.int64)
    lab[:, :12] = 0
    filters = O.expand_bank(O.paper_bank(36, 36, "23rect", 1))
    r = O.template_representation(lab, 2, filters)
    e8, e4 = math.exp(-1 / 8), math.exp(-1 / 4)
    left = (2 * e4 + e8) / 9.0             # sum of a Gaussian column at the edge, / 9
    mid = (2 * e8 + 1.0) / 9.0
    # gauss, haar2x, haar2y, haar3x, haar3y; channels (0, 1)
    expect = [[left, left + mid],
              [left, -left],
              [0.0, 0.0],                                  # rows weigh +1, 0, -1: symmetric columns cancel
              [left, -2 * mid + left],
              [(2 * e4 - 2 * e8) / 9.0, (2 * e4 - 2) / 9.0]]  # rows weigh +1, -2, +1
    np.testing.assert_allclose(r, np.array(expect), rtol=1e-14, atol=1e-15)


def _sim(tl, ql, k, bank):
    filters = O.expand_bank(bank)
    rt = O.template_representation(tl, k, filters)
    h, w = tl.shape
    return O.similarity_map_fast(ql, k, w, h, filters, rt)


def test_mirror_and_transpose_symmetry():
    """36 x 36 template, scales 1..3: every sub-window is centred exactly and
    split into equal thirds, so mirroring template and query left-right negates
    each Haar-x response on both sides (|R_t - R_q| unchanged) and keeps the
    others; transposing swaps the x and y filters, which share a weight."""
    rng = np.random.default_rng(11)
    k = 6
    ql = rng.integers(0, k, size=(50, 44))
    tl = rng.integers(0, k, size=(36, 36))
    bank = O.paper_bank(36, 36, "23rect", 3)
    s0 = _sim(tl, ql, k, bank)
    s1 = _sim(tl[:, ::-1], ql[:, ::-1], k, bank)
    np.testing.assert_allclose(s1[:, ::-1], s0, rtol=1e-12, atol=1e-14)
    s2 = _sim(tl.T.copy(), ql.T.copy(), k, bank)
    np.testing.assert_allclose(s2.T, s0, rtol=1e-12, atol=1e-14)
    # a left-right mix-up in the Haar-x filters would break the first identity on
    # a template that is not mirror-symmetric; make sure the test can see it
    assert not np.allclose(_sim(tl[:, ::-1], ql, k, bank), s0)


def test_noise_free_crop_scores_zero_with_the_paper_bank():
    rng = np.random.default_rng(12)
    k = 8
    ql = rng.integers(0, k, size=(64, 72))
    x0, y0, w, h = 17, 9, 30, 27
    tl = ql[y0:y0 + h, x0:x0 + w].copy()
    s = _sim(tl, ql, k, O.paper_bank(w, h, "23rect", 3))
    assert s[y0, x0] == 0.0
    assert O.localise(s)[:2] == (x0, y0)
    assert np.all(s <= 0.0)


def test_loop_and_vectorised_similarity_agree_on_weighted_banks():
    rng = np.random.default_rng(13)
    k = 5
    ql = rng.integers(0, k, size=(30, 33))
    tl = rng.integers(0, k, size=(14, 17))
    filters = O.expand_bank(O.paper_bank(17, 14, "23rect", 2))
    rt = O.template_representation(tl, k, filters)
    a = O.similarity_map(ql, k, 17, 14, filters, rt)
    b = O.similarity_map_fast(ql, k, 17, 14, filters, rt)
    assert np.array_equal(a, b)
