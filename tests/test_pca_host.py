"""The library's PCA fit (host: FP64 covariance, subspace iteration) against
the oracle's (numpy eigh), on the host: same mean, same axes (each up to the
sign convention both apply), same variances, within the accuracy of an
FP32 result; argument errors."""
import numpy as np
import pytest

from oracle import vqnnf_oracle as O
from paper_2306_15010_amd import binding as B
from paper_2306_15010_amd import synth


def _planted(h, w, D, seed):
    rng = np.random.default_rng(seed)
    n = h * w
    axes = np.linalg.qr(rng.standard_normal((D, 4)))[0].T
    g = rng.standard_normal((n, 4))
    g -= g.mean(axis=0)
    coef = np.linalg.qr(g)[0] * np.sqrt(n) * np.array([5.0, 3.0, 2.0, 1.0])
    x = 0.7 + coef @ axes + 0.01 * rng.standard_normal((n, D))
    return x.reshape(h, w, D).astype(np.float32)


@pytest.mark.parametrize("h,w,D,d,seed", [(40, 40, 64, 4, 1), (30, 50, 128, 3, 2), (25, 25, 24, 2, 3)])
def test_pca_fit_matches_oracle(h, w, D, d, seed):
    t = _planted(h, w, D, seed)
    mean, basis, var = B.vqnnf_pca_fit(t, d)
    om, ob, ov = O.pca_fit(t.reshape(-1, D).astype(np.float64), d)
    np.testing.assert_allclose(mean, om, rtol=0, atol=1e-6)
    np.testing.assert_allclose(basis, ob, rtol=0, atol=2e-6)
    np.testing.assert_allclose(var, ov, rtol=2e-6)


def test_pca_fit_mixture_features_and_rgb():
    # the smooth-mixture features of the benchmark maps: leading axes separated
    t = synth.random_map(48, 48, 64, "f32", seed=9, M=24).data
    x = t.reshape(-1, 64).astype(np.float64)
    om, ob, ov = O.pca_fit(x, 9)
    assert np.all(ov[:-1] / ov[1:] > 1.01)          # distinct variances: axes well defined
    mean, basis, var = B.vqnnf_pca_fit(t, 9)
    np.testing.assert_allclose(basis, ob, rtol=0, atol=5e-5)
    np.testing.assert_allclose(var, ov, rtol=1e-5)
    # colour features of an RGB template
    img = synth.rgb_image(30, 30, seed=4)
    mean, basis, var = B.vqnnf_pca_fit(img, 5)
    om, ob, ov = O.pca_fit(O.rgb_patch_features(img).reshape(-1, 27), 5)
    np.testing.assert_allclose(mean, om, rtol=1e-6)
    np.testing.assert_allclose(var, ov, rtol=1e-5)
    for r in range(5):
        assert abs(abs(float(basis[r] @ ob[r])) - 1.0) < 1e-4


def test_pca_argument_errors():
    t = synth.random_map(8, 8, 6, "f32", seed=1).data
    for d in (0, 7, 65):
        with pytest.raises(B.VqnnfError) as ei:
            B.vqnnf_pca_fit(t, d)
        assert ei.value.status == B.VQNNF_EINVAL
    ctx = B.Context(host=True)

    class Fake:
        def data_ptr(self):
            return 0x1000

    q = B.FMap(0x1000, B.VQNNF_BF16, 16, 16, 6, 6, None)
    with pytest.raises(B.VqnnfError) as ei:
        B.vqnnf_pca_project(ctx, q, np.zeros(6), np.zeros((2, 6)), Fake())
    assert ei.value.status == B.VQNNF_ENOTSUP       # valid arguments, no device
    with pytest.raises(B.VqnnfError) as ei:
        B.vqnnf_pca_project(ctx, q, np.zeros(6), np.full((2, 6), np.nan), Fake())
    assert ei.value.status == B.VQNNF_EINVAL
