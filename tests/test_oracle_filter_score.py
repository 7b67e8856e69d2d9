"""Pins for the oracle's integral image (O4), filters (O5), template
representation (O6), similarity (O7) and localisation (O8)."""
import numpy as np
import pytest

from oracle import vqnnf_oracle as O
from paper_2306_15010_amd import synth


def _labels(H, W, k, seed):
    return np.random.default_rng(seed).integers(0, k, size=(H, W))


# ------------------------------------------------------------------ O4

def test_integral_matches_direct_counts():
    lab = _labels(7, 9, 4, 0)
    P = O.integral_image(lab, 4)
    assert P.shape == (8, 10, 4)
    for y in range(8):
        for x in range(10):
            direct = np.bincount(lab[:y, :x].reshape(-1), minlength=4) if x and y else np.zeros(4)
            assert np.array_equal(P[y, x], direct)


def test_integral_invariants():
    lab = _labels(13, 11, 5, 1)
    P = O.integral_image(lab, 5)
    assert P[13, 11].sum() == 13 * 11
    assert np.all(P[0] == 0) and np.all(P[:, 0] == 0)
    assert np.all(np.diff(P, axis=0) >= 0) and np.all(np.diff(P, axis=1) >= 0)
    # each 2x2 difference is the one-hot of the pixel
    d = P[1:, 1:] - P[:-1, 1:] - P[1:, :-1] + P[:-1, :-1]
    assert np.array_equal(d, O.one_hot(lab, 5))


def test_paper_inclusive_form_and_box_sum():
    lab = _labels(6, 8, 3, 2)
    P = O.integral_image(lab, 3)
    for y in range(6):
        for x in range(8):
            incl = np.zeros(3, dtype=np.int64)
            for yy in range(y + 1):
                for xx in range(x + 1):
                    incl[lab[yy, xx]] += 1
            assert np.array_equal(P[y + 1, x + 1], incl)
    rng = np.random.default_rng(3)
    for _ in range(50):
        x0, x1 = sorted(rng.integers(0, 9, size=2))
        y0, y1 = sorted(rng.integers(0, 7, size=2))
        ref = np.bincount(lab[y0:y1, x0:x1].reshape(-1), minlength=3)
        assert np.array_equal(O.box_sum(P, x0, y0, x1, y1), ref)


def test_window_histograms_sum_to_area():
    lab = _labels(20, 24, 6, 4)
    P = O.integral_image(lab, 6)
    w, h = 7, 5
    for y in range(20 - h + 1):
        for x in range(24 - w + 1):
            assert O.box_sum(P, x, y, x + w, y + h).sum() == w * h


# ------------------------------------------------------------------ O5

@pytest.mark.parametrize("n,g,edges", [(16, 2, [0, 8, 16]), (25, 3, [0, 8, 16, 25]),
                                       (96, 3, [0, 32, 64, 96]), (7, 1, [0, 7])])
def test_grid_edges(n, g, edges):
    assert O.grid_edges(0, n, g) == edges


def test_bins_partition_the_window():
    lab = _labels(30, 30, 5, 5)
    P = O.integral_image(lab, 5)
    filters = O.expand_bank(O.default_bank(17, 13, 3))
    assert len(filters) == 10
    for (x, y) in [(0, 0), (5, 9), (13, 17)]:
        r = O.filter_responses(P, x, y, filters)
        assert np.array_equal(r[1:].sum(axis=0), r[0])
        assert np.array_equal(r[0], np.bincount(lab[y:y + 13, x:x + 17].reshape(-1), minlength=5))


def test_default_weights_normalise_each_term():
    filters = O.expand_bank(O.default_bank(25, 25, 3))
    assert filters[0].weight == 1.0 / 625
    edges = O.grid_edges(0, 25, 3)
    areas = [(edges[a + 1] - edges[a]) * (edges[b + 1] - edges[b]) for b in range(3) for a in range(3)]
    for f, area in zip(filters[1:], areas):
        assert f.weight == 1.0 / (9 * area)


def test_alg2_dilation_equals_direct_weighted_bins():
    rng = np.random.default_rng(6)
    lab = _labels(40, 40, 4, 7)
    P = O.integral_image(lab, 4)
    for rh, rw in [(3, 3), (2, 4), (1, 1), (3, 2)]:
        f = rng.standard_normal((rh, rw))
        fd = O.dilation_filter(f)
        assert fd.shape == (rh + 1, rw + 1)
        w, h = 23, 19
        xs, ys = O.grid_edges(0, w, rw), O.grid_edges(0, h, rh)
        for (x, y) in [(0, 0), (3, 11), (17, 21)]:
            direct = np.zeros(4)
            for b in range(rh):
                for a in range(rw):
                    sub = lab[y + ys[b]:y + ys[b + 1], x + xs[a]:x + xs[a + 1]]
                    direct += f[b, a] * np.bincount(sub.reshape(-1), minlength=4)
            np.testing.assert_allclose(O.dilated_response(P, x, y, fd, xs, ys), direct,
                                       rtol=1e-12, atol=1e-9)


def test_alg2_single_bin_is_the_box_sum():
    fd = O.dilation_filter(np.ones((1, 1)))
    assert np.array_equal(fd, np.array([[1.0, -1.0], [-1.0, 1.0]]))


def test_rot90_permutes_bins_and_keeps_full_window():
    rng = np.random.default_rng(8)
    tl = rng.integers(0, 6, size=(12, 12))
    filters = O.expand_bank(O.default_bank(12, 12, 3))
    r0 = O.template_representation(tl, 6, filters)
    r1 = O.template_representation(np.rot90(tl), 6, filters)
    assert np.array_equal(r0[0], r1[0])
    assert sorted(map(tuple, r0[1:])) == sorted(map(tuple, r1[1:]))


# ------------------------------------------------------------------ O7 / O8

def test_noise_free_crop_scores_zero_and_is_the_maximum():
    rng = np.random.default_rng(9)
    q = rng.standard_normal((40, 44, 5))
    x0, y0, w, h = 17, 9, 12, 10
    t = q[y0:y0 + h, x0:x0 + w].astype(np.float32)
    q32 = q.astype(np.float32).astype(np.float64)
    res = O.match(t, q32, 6, O.default_bank(w, h, 2), iters=10, seed=3)
    assert res.sim.shape == (40 - h + 1, 44 - w + 1)
    assert res.sim[y0, x0] == 0.0
    assert np.all(res.sim <= 0.0) and np.all(res.sim >= -4.0)
    bx, by, bs = res.best
    assert bs == 0.0 and res.sim[by, bx] == 0.0


def test_fast_and_per_window_similarity_agree_and_match_bruteforce():
    rng = np.random.default_rng(10)
    k, w, h = 5, 9, 7
    ql = rng.integers(0, k, size=(20, 23))
    tl = rng.integers(0, k, size=(h, w))
    filters = O.expand_bank(O.default_bank(w, h, 3))
    rt = O.template_representation(tl, k, filters)
    fast = O.similarity_map_fast(ql, k, w, h, filters, rt)
    slow = O.similarity_map(ql, k, w, h, filters, rt)
    assert np.array_equal(fast, slow)
    xs, ys = O.grid_edges(0, w, 3), O.grid_edges(0, h, 3)
    regions = [(0, 0, w, h)] + [(xs[a], ys[b], xs[a + 1], ys[b + 1]) for b in range(3) for a in range(3)]
    for (x, y) in [(0, 0), (4, 6), (14, 13)]:
        s = 0.0
        for i, (rx0, ry0, rx1, ry1) in enumerate(regions):
            ht = np.bincount(tl[ry0:ry1, rx0:rx1].reshape(-1), minlength=k)
            hq = np.bincount(ql[y + ry0:y + ry1, x + rx0:x + rx1].reshape(-1), minlength=k)
            area = (rx1 - rx0) * (ry1 - ry0)
            wt = 1.0 / area if i == 0 else 1.0 / (9 * area)
            s += wt * np.abs(ht - hq).sum()
        assert fast[y, x] == pytest.approx(-s, rel=1e-14, abs=1e-15)


def test_localise_row_major_tie_break():
    s = np.full((4, 5), -1.0)
    s[2, 1] = s[1, 3] = s[3, 0] = 0.5
    assert O.localise(s) == (3, 1, 0.5)


def test_c1_shape_and_planted_offset_found():
    found = 0
    for seed in range(4):
        wl = synth.make_config("c1", seed=synth.MASTER_SEED + 1000 * seed)
        qm, t = wl.maps[0], wl.templates[0][0]
        q = O.decode(qm.dtype, qm.data, qm.scale)
        res = O.match(t.data, q, t.k, O.default_bank(16, 16, t.grid), seed=seed)
        assert res.sim.shape == (49, 49)
        bx, by, _ = res.best
        found += (bx, by) == (t.x0, t.y0)
    assert found >= 3
