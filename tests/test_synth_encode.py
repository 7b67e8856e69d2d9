"""The input generator's FP8 E4M3FN encoder: the integer form used for
generation gives the same codes as the frexp form on grid values, midpoints,
their neighbours and random values over the whole range; every finite code
round-trips; ties go to the even code; values beyond 448 saturate."""
import numpy as np

from oracle import vqnnf_oracle as O
from paper_2306_15010_amd import synth as S


def test_encoder_forms_agree():
    rng = np.random.default_rng(0)
    vals = S._E4M3_POS.astype(np.float64)
    mids = (vals[1:] + vals[:-1]) / 2
    c = np.concatenate([vals, mids, [448.0, 464.0, 480.0, 1e4, 2.0 ** -6, 2.0 ** -10, 0.0]])
    c = np.concatenate([c, np.nextafter(c, np.inf), np.nextafter(c, -np.inf)])
    c = np.concatenate([c, -c, rng.standard_normal(200_000) * 100, rng.uniform(-1, 1, 200_000) * 2.0 ** -5,
                        np.exp(rng.uniform(-30, 7, 200_000))])
    assert np.array_equal(S.f32_to_e4m3fn(c), S.f32_to_e4m3fn_frexp(c))


def test_encoder_round_trip_ties_and_saturation():
    codes = np.array([c for c in range(256) if c & 0x7F != 0x7F], dtype=np.uint8)
    v = np.array([O.e4m3fn_value(int(c)) for c in codes])
    enc = S.f32_to_e4m3fn(v)
    # +0 and -0 both encode to code 0
    assert np.array_equal(np.where(v == 0, 0, enc), np.where(v == 0, 0, codes))
    pos = S._E4M3_POS.astype(np.float64)
    mids = (pos[1:] + pos[:-1]) / 2
    e = S.f32_to_e4m3fn(mids)
    lo = np.arange(len(mids))
    # a midpoint goes to whichever neighbour has the even code
    assert np.array_equal(e, np.where(lo % 2 == 0, lo, lo + 1).astype(np.uint8))
    assert S.f32_to_e4m3fn(np.array([449.0, 1e30, -500.0])).tolist() == [0x7E, 0x7E, 0xFE]
