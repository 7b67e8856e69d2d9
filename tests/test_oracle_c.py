"""Pins for the C variant of the FP64 oracle: every function returns the
Python oracle's values bit for bit (decode, FP64 distances, labels, k-means
codebooks in FP64 and FP32), and the generator and the k-means++ draw rule are
pinned by hand-computed cases from the generator's published outputs.

The Python oracle is pinned against the paper and the mathematics in the
other oracle tests; this file ties the C variant (used where the Python one
is too slow: full-size label maps) to it."""
import numpy as np
import pytest

from oracle import vqnnf_oracle as O
from oracle import vqnnf_oracle_c as OC
from paper_2306_15010_amd import synth

# First outputs of Vigna's splitmix64 from seed 0 (published test values).
SM_SEED0 = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def _bits(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


def test_splitmix64_and_u01_hand_values():
    out, u = OC.splitmix64(0, 3)
    assert [int(v) for v in out] == SM_SEED0
    # u01 keeps the top 53 bits: (x >> 11) * 2^-53, computed here by hand
    for x, v in zip(SM_SEED0, u):
        assert v == (x >> 11) / 2.0 ** 53
    g = O.SplitMix64(0)
    assert [g.u01() for _ in range(3)] == [(x >> 11) / 2.0 ** 53 for x in SM_SEED0]
    # a low-bits variant would differ on the first output
    assert (SM_SEED0[0] >> 11) != (SM_SEED0[0] & (2 ** 53 - 1))


def test_kmeanspp_four_point_draw_by_hand():
    """Points 0, 1, 3, 7 on a line, seed 0, k = 2, no Lloyd iteration.
    u0 = 0xE220A8397B1DCDAF >> 11 times 2^-53 = 0.8833...: first centre
    index floor(4 u0) = 3 (the point 7).  D^2 = 49, 36, 16, 0, S = 101;
    u1 = 0x6E789E6AA1B965F4 >> 11 times 2^-53 = 0.4315...: target 43.58...,
    running sums 49, 85, 101, 101: the first above it is index 0 (point 0)."""
    u0 = (SM_SEED0[0] >> 11) / 2.0 ** 53
    u1 = (SM_SEED0[1] >> 11) / 2.0 ** 53
    assert int(u0 * 4) == 3 and 36.0 < u1 * 101.0 < 49.0
    t = np.array([0.0, 1.0, 3.0, 7.0], dtype=np.float32).reshape(1, 4, 1)
    for cb in (O.kmeans_codebook(t, 2, 0, seed=0), OC.kmeans_codebook(t, 2, 0, seed=0)):
        assert cb[:, 0].tolist() == [7.0, 0.0]
    # one Lloyd step: clusters {7} and {0, 1, 3}
    for cb in (O.kmeans_codebook(t, 2, 1, seed=0), OC.kmeans_codebook(t, 2, 1, seed=0)):
        assert cb[:, 0].tolist() == [7.0, np.float32(4.0 / 3.0)]


class _FixedU:
    """A stand-in generator returning chosen u values."""

    def __init__(self, us):
        self.us = list(us)

    def u01(self):
        return self.us.pop(0)


def test_kmeanspp_draw_is_strictly_greater():
    """D^2 = 16, 16, 0, 32 after the first centre (S = 64) and u = 1/4:
    target 16 equals the first running sum exactly; the rule takes the first
    running sum *strictly* above it, index 1 (a >= rule would take 0)."""
    x = np.array([[4.0, 0.0], [-4.0, 0.0], [0.0, 0.0], [4.0, 4.0]])
    # first centre: u = 0.5 -> index 2 (the origin); D^2 exact integers
    c = O.kmeans_pp_init(x, 2, _FixedU([0.5, 0.25]))
    assert c[0].tolist() == [0.0, 0.0] and c[1].tolist() == [-4.0, 0.0]
    # u just below 1/4 -> target below 16 -> index 0
    c = O.kmeans_pp_init(x, 2, _FixedU([0.5, 0.25 - 2.0 ** -54]))
    assert c[1].tolist() == [4.0, 0.0]


def test_decode_matches_python_oracle():
    b = np.arange(65536, dtype=np.uint16)
    ref, got = O.decode("bf16", b), OC.decode("bf16", b[:, None])[:, 0]
    fin = np.isfinite(ref)
    assert np.array_equal(_bits(ref[fin]), _bits(got[fin])) and np.array_equal(fin, np.isfinite(got))
    codes = np.arange(256, dtype=np.uint8)
    for s in (1.0, 0.0078125, 3.3e-3, 1.7e4):
        scale = np.array([s], dtype=np.float32)
        ref = O.decode("fp8", codes[:, None], scale)[:, 0]
        got = OC.decode("fp8", codes[:, None], scale)[:, 0]
        fin = np.isfinite(ref)
        assert np.array_equal(_bits(ref[fin]), _bits(got[fin])) and np.array_equal(fin, np.isfinite(got))
    assert all(OC.e4m3fn_value(c) == O.e4m3fn_value(c) for c in range(256) if c & 0x7F != 0x7F)
    x = np.random.default_rng(1).standard_normal((50, 7)).astype(np.float32)
    assert np.array_equal(_bits(O.decode("f32", x)), _bits(OC.decode("f32", x)))


@pytest.mark.parametrize("dtype,D,k,seed", [("f32", 27, 8, 1), ("bf16", 64, 32, 2), ("fp8", 64, 16, 3),
                                            ("bf16", 512, 128, 4), ("f32", 5, 1, 5), ("fp8", 33, 256, 6)])
def test_distances_and_labels_match_python_oracle(dtype, D, k, seed):
    qm = synth.random_map(13, 11, D, dtype, seed=seed)
    rng = np.random.default_rng(seed)
    cb = (qm.decoded_f32().reshape(-1, D)[rng.integers(0, 143, size=k)]
          + 0.05 * rng.standard_normal((k, D))).astype(np.float32).astype(np.float64)
    q = O.decode(dtype, qm.data, qm.scale).reshape(-1, D)
    ref = O.sq_distances(q, cb)
    for nt in (1, 3):
        got = OC.sq_distances_map(dtype, qm.data, qm.scale, cb, n_threads=nt)
        assert np.array_equal(_bits(ref), _bits(got))
        lab = OC.assign_map(dtype, qm.data, qm.scale, cb, n_threads=nt)
        assert np.array_equal(lab.reshape(-1).astype(np.int64), O.assign(q, cb))


def test_labels_tie_to_lowest_index():
    # duplicate codewords and exact dyadic midpoints
    cb = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 0.0], [0.5, 0.0]])
    q = np.array([[0.75, 0.0], [0.25, 0.0], [1.0, 0.0], [2.0, 0.0]], dtype=np.float32)
    lab = OC.assign_map("f32", q, None, cb)
    assert lab.tolist() == O.assign(q.astype(np.float64), cb).tolist() == [1, 0, 1, 1]


@pytest.mark.parametrize("shape,k,iters,seed", [((8, 8, 3), 5, 20, 0), ((12, 9, 27), 8, 20, 7),
                                                ((6, 7, 64), 32, 20, 3), ((10, 10, 512), 16, 4, 11),
                                                ((3, 4, 6), 12, 20, 5), ((5, 5, 4), 9, 3, 2)])
def test_kmeans_matches_python_oracle(shape, k, iters, seed):
    rng = np.random.default_rng(seed)
    t = rng.standard_normal(shape).astype(np.float32)
    if seed == 2:      # duplicated points: zero D^2 sums and empty clusters
        t[:, :3] = t[0, 0]
    c32, c64 = O.kmeans_codebook(t, k, iters, seed=seed, return_f64=True)
    for nt in (1, 4):
        g32, g64 = OC.kmeans_codebook(t, k, iters, seed=seed, return_f64=True, n_threads=nt)
        assert np.array_equal(_bits(c64), _bits(g64))
        assert np.array_equal(c32.view(np.uint32), g32.view(np.uint32))


def test_kmeans_identical_points():
    t = np.tile(np.array([0.25, -1.0, 3.0], dtype=np.float32), (4, 5, 1))
    assert np.all(OC.kmeans_codebook(t, 4, 5, seed=1) == t[0, 0])
