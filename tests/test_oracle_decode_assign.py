"""Pins for the oracle's decode (O1) and nearest-codeword assignment (O3).

Each check ties the oracle to something other than its own formula: values
fixed by the storage formats, an independent library decoder, exact rational
arithmetic, or constructed cases whose answer is known in closed form.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import vqnnf_oracle as O


# ------------------------------------------------------------------ O1 decode

def test_bf16_known_values():
    bits = np.array([0x0000, 0x8000, 0x3F80, 0xC000, 0x4049, 0x0001, 0x7F7F, 0x0080],
                    dtype=np.uint16)
    v = O.decode_bf16(bits)
    assert v[0] == 0.0 and math.copysign(1, v[1]) < 0
    assert v[2] == 1.0 and v[3] == -2.0
    assert v[4] == 3.140625                       # 0x4049 = 1.5703125 * 2
    assert v[5] == 2.0 ** -133                    # smallest subnormal
    assert v[6] == (2 - 2 ** -7) * 2.0 ** 127     # largest finite
    assert v[7] == 2.0 ** -126                    # smallest normal


def test_bf16_exhaustive_against_field_formula():
    bits = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    v = O.decode_bf16(bits)
    for b in range(0, 65536, 7):
        s, e, m = b >> 15, (b >> 7) & 0xFF, b & 0x7F
        if e == 0xFF:
            assert not np.isfinite(v[b])
            continue
        ref = math.ldexp(m, -133) if e == 0 else math.ldexp(128 + m, e - 134)
        assert v[b] == (-ref if s else ref)


def test_e4m3fn_known_values():
    t = O.E4M3FN_TABLE
    assert t[0x00] == 0.0
    assert t[0x38] == 1.0 and t[0xB8] == -1.0
    assert t[0x7E] == 448.0 and t[0xFE] == -448.0       # largest finite
    assert t[0x08] == 2.0 ** -6                         # smallest normal
    assert t[0x01] == 2.0 ** -9                         # smallest subnormal
    assert t[0x07] == 7 * 2.0 ** -9
    assert math.isnan(t[0x7F]) and math.isnan(t[0xFF])
    assert np.all(np.isfinite(np.delete(t, [0x7F, 0xFF])))


def test_e4m3fn_exhaustive_against_torch():
    torch = pytest.importorskip("torch")
    codes = torch.arange(256, dtype=torch.int32).to(torch.uint8)
    ref = codes.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    t = O.E4M3FN_TABLE
    nan = np.isnan(ref)
    assert np.array_equal(nan, np.isnan(t))
    assert np.array_equal(ref[~nan], t[~nan])


def test_fp8_scaled_decode_is_exact():
    rng = np.random.default_rng(1)
    codes = rng.integers(0, 256, size=400).astype(np.uint8)
    codes[(codes & 0x7F) == 0x7F] = 0x11
    scale = rng.uniform(1e-3, 3.0, size=400).astype(np.float32)
    v = O.decode_e4m3fn(codes, scale)
    for c, s, x in zip(codes, scale, v):
        exact = Fraction(float(s)) * Fraction(O.e4m3fn_value(int(c)))
        assert Fraction(float(x)) == exact


# ------------------------------------------------------------------ O3 assign

def _exact_sqdist(p, c):
    return sum((Fraction(float(a)) - Fraction(float(b))) ** 2 for a, b in zip(p, c))


def test_assign_matches_exact_rational_bruteforce():
    rng = np.random.default_rng(7)
    checked = 0
    for trial in range(30):
        D = int(rng.integers(1, 9))
        k = int(rng.integers(1, 7))
        n = 25
        x = rng.standard_normal((n, D)).astype(np.float32).astype(np.float64)
        c = rng.standard_normal((k, D)).astype(np.float32).astype(np.float64)
        lab = O.assign(x, c)
        d64 = O.sq_distances(x, c)
        for p in range(n):
            ex = [_exact_sqdist(x[p], c[j]) for j in range(k)]
            best = min(range(k), key=lambda j: (ex[j], j))
            others = [ex[j] for j in range(k) if j != best]
            gap = min(others) - ex[best] if others else Fraction(1)
            # FP64 rounding of a distance is below (D+2)*2^-53 relative
            e64 = Fraction(D + 2, 2 ** 52) * max(ex)
            if gap > 2 * e64:
                assert lab[p] == best
                checked += 1
            for j in range(k):
                assert abs(Fraction(float(d64[p, j])) - ex[j]) <= e64
    assert checked > 600


def test_assign_exact_tie_goes_to_lowest_index():
    # dyadic codewords and their exact midpoints: equal distances, exact in FP64
    c = np.array([[0.5, -1.25, 2.0], [1.5, 0.75, -2.0], [0.5, -1.25, 2.0]])
    mid = (c[0] + c[1]) / 2
    x = np.stack([mid, c[2], c[1]])
    lab = O.assign(x, c)
    assert lab[0] == 0          # tie between 0 and 1
    assert lab[1] == 0          # duplicate codewords 0 and 2: lowest wins
    assert lab[2] == 1          # exact hit


def test_assign_single_codeword():
    x = np.random.default_rng(0).standard_normal((50, 5))
    assert np.all(O.assign(x, x[:1]) == 0)


def test_assign_follows_sequential_fp64_order():
    """The distance order is part of the contract: sequential in t from 0,
    with no FMA.  Codeword 0's terms are 1 then four 2^-54: a running sum
    stays at 1 (2^-54 is below half an ulp of 1, so each add rounds back),
    while exact or pairwise summation gives 1 + 2^-52.  Codeword 1 is at distance exactly 1.
    Under the sequential contract the two tie and the lower index wins."""
    q = np.zeros((1, 5))
    c = np.array([[1.0, 2 ** -27, 2 ** -27, 2 ** -27, 2 ** -27],
                  [1.0, 0.0, 0.0, 0.0, 0.0]])
    d = O.sq_distances(q, c)
    assert d[0, 0] == 1.0 and d[0, 1] == 1.0
    assert O.assign(q, c)[0] == 0
    # reversed order of the same terms would be caught: pairwise gives more
    assert (2 ** -54 + 2 ** -54) + (2 ** -54 + 2 ** -54) + 1.0 == 1.0 + 2 ** -52


# ------------------------------------------------------------------ colour patches (Sec. 5.2)

def test_rgb_patch_features_by_hand():
    """2 x 3 image with distinct channel values; every feature of two pixels
    written out from the definition (3x3 neighbourhood, edge replication)."""
    img = np.arange(2 * 3 * 3, dtype=np.uint8).reshape(2, 3, 3) * 7
    f = O.rgb_patch_features(img)
    assert f.shape == (2, 3, 27)
    # pixel (x=1, y=0): rows y-1 -> 0 (replicated), 0, 1; columns 0, 1, 2
    expect = []
    for yy in (0, 0, 1):
        for xx in (0, 1, 2):
            expect += [int(v) for v in img[yy, xx]]
    assert f[0, 1].tolist() == expect
    # corner pixel (x=2, y=1): rows 0, 1, 1; columns 1, 2, 2
    expect = []
    for yy in (0, 1, 1):
        for xx in (1, 2, 2):
            expect += [int(v) for v in img[yy, xx]]
    assert f[1, 2].tolist() == expect
    # the centre of each patch is the pixel itself
    assert np.array_equal(f[:, :, 12:15], img.astype(np.float64))


def test_rgb_patch_features_invariants():
    rng = np.random.default_rng(3)
    img = rng.integers(0, 256, size=(9, 11, 3)).astype(np.uint8)
    f = O.rgb_patch_features(img)
    # interior pixel: feature block (dy, dx) is the pixel at (x+dx-1, y+dy-1)
    for dy in range(3):
        for dx in range(3):
            assert np.array_equal(f[1:-1, 1:-1, (3 * dy + dx) * 3:(3 * dy + dx) * 3 + 3],
                                  img[dy:dy + 7, dx:dx + 9].astype(np.float64))
    # a constant image gives identical features everywhere
    c = np.full((4, 5, 3), 17, np.uint8)
    assert np.all(O.rgb_patch_features(c) == 17)
    assert np.array_equal(O.decode("rgb8", img), f)
