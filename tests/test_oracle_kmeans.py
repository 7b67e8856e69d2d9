"""Pins for the oracle's k-means codebook (O2)."""
import numpy as np

from oracle import vqnnf_oracle as O


def test_splitmix64_reference_outputs():
    # First outputs of Vigna's splitmix64 for seed 0.
    g = O.SplitMix64(0)
    assert g.next() == 0xE220A8397B1DCDAF
    assert g.next() == 0x6E789E6AA1B965F4
    assert g.next() == 0x06C45D188009454F


def test_u01_range_and_resolution():
    g = O.SplitMix64(123)
    u = [g.u01() for _ in range(1000)]
    assert min(u) >= 0.0 and max(u) < 1.0
    for v in u:
        assert v * 2 ** 53 == int(v * 2 ** 53)


def test_k_equals_points_gives_the_points():
    rng = np.random.default_rng(3)
    t = rng.standard_normal((3, 4, 6)).astype(np.float32)
    cb = O.kmeans_codebook(t, 12, 20, seed=5)
    pts = t.reshape(-1, 6)
    key = lambda a: sorted(map(tuple, a.tolist()))
    assert key(cb) == key(pts)


def test_identical_points_give_that_point():
    t = np.tile(np.array([0.25, -1.0, 3.0], dtype=np.float32), (4, 5, 1))
    cb = O.kmeans_codebook(t, 4, 5, seed=1)
    assert np.all(cb == t[0, 0])


def test_two_separated_blobs_give_blob_means():
    rng = np.random.default_rng(11)
    a = rng.normal(-10.0, 0.5, size=(40, 3))
    b = rng.normal(+10.0, 0.5, size=(24, 3))
    pts = np.concatenate([a, b]).astype(np.float32)
    t = pts.reshape(8, 8, 3)
    cb = O.kmeans_codebook(t, 2, 20, seed=9)
    cb = cb[np.argsort(cb[:, 0])]
    ma = a.astype(np.float32).astype(np.float64).mean(axis=0)
    mb = b.astype(np.float32).astype(np.float64).mean(axis=0)
    np.testing.assert_allclose(cb[0], ma, rtol=1e-6)
    np.testing.assert_allclose(cb[1], mb, rtol=1e-6)


def test_lloyd_objective_never_increases_and_is_fixed_point():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((300, 5))
    c0 = O.kmeans_pp_init(x, 7, O.SplitMix64(2))
    hist = []
    c = O.lloyd(x, c0, 30, history=hist)
    assert all(hist[i + 1] <= hist[i] * (1 + 1e-12) for i in range(len(hist) - 1))
    lab = O.assign(x, c)
    for j in range(7):
        pts = x[lab == j]
        if len(pts):
            np.testing.assert_allclose(c[j], pts.mean(axis=0), rtol=1e-9, atol=1e-12)


def test_kmeanspp_draws_only_where_distance_is_positive():
    # all points coincide except one: once the first centre is chosen the
    # only point with D^2 > 0 (or the duplicate cluster) must come next
    x = np.zeros((10, 2))
    x[7] = [5.0, 5.0]
    for seed in range(20):
        c = O.kmeans_pp_init(x, 2, O.SplitMix64(seed))
        assert {tuple(c[0]), tuple(c[1])} == {(0.0, 0.0), (5.0, 5.0)}


def test_kmeanspp_first_centre_uniform_index():
    x = np.arange(10, dtype=np.float64)[:, None]
    g = O.SplitMix64(42)
    u = O.SplitMix64(42).u01()
    c = O.kmeans_pp_init(x, 1, g)
    assert c[0, 0] == int(u * 10)
