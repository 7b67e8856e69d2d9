"""Pins for the oracle's PCA reduction (O1b, Sec. 5.5): properties PCA has by
definition, checked on data whose principal structure is planted, so that a
transposed basis, a missing centring or a wrong ordering fails."""
import numpy as np

from oracle import vqnnf_oracle as O


def _planted(n=4000, D=24, seed=0):
    """Points on a planted 3-D subspace with variances 9, 4, 1 (orthonormal
    axes), offset by a mean, plus tiny isotropic noise."""
    rng = np.random.default_rng(seed)
    axes = np.linalg.qr(rng.standard_normal((D, 3)))[0].T          # 3 orthonormal rows
    # coefficient columns with zero mean, exactly orthogonal, of variance 9, 4, 1
    g = rng.standard_normal((n, 3))
    g -= g.mean(axis=0)
    coef = np.linalg.qr(g)[0] * np.sqrt(n) * np.array([3.0, 2.0, 1.0])
    mu = rng.standard_normal(D) * 5
    x = mu + coef @ axes + 1e-6 * rng.standard_normal((n, D))
    return x, axes, mu, coef


def test_pca_recovers_planted_axes_and_variances():
    x, axes, mu, coef = _planted()
    mean, basis, var = O.pca_fit(x, 3)
    np.testing.assert_allclose(mean, x.mean(axis=0), rtol=0, atol=1e-12)
    # each fitted axis is a planted axis up to sign, in decreasing variance
    for r in range(3):
        assert abs(abs(basis[r] @ axes[r]) - 1.0) < 1e-8
    np.testing.assert_allclose(var, [9.0, 4.0, 1.0], rtol=1e-6)
    assert var[0] > var[1] > var[2]


def test_pca_projection_decorrelates_and_reconstructs():
    rng = np.random.default_rng(1)
    D = 10
    x = rng.standard_normal((500, D)) @ rng.standard_normal((D, D))
    mean, basis, var = O.pca_fit(x, D)
    y = O.pca_project(x, mean, basis)
    cov = (y.T @ y) / len(y)
    np.testing.assert_allclose(cov, np.diag(var), atol=1e-9 * var[0])
    # full rank: the basis is orthonormal and projection is invertible
    np.testing.assert_allclose(basis @ basis.T, np.eye(D), atol=1e-12)
    np.testing.assert_allclose(y @ basis + mean, x, atol=1e-9)


def test_pca_sign_convention_and_prefix():
    x, _, _, _ = _planted(seed=2)
    _, b3, _ = O.pca_fit(x, 3)
    _, b2, _ = O.pca_fit(x, 2)
    np.testing.assert_array_equal(b2, b3[:2])            # d only truncates
    for r in range(3):
        j = int(np.argmax(np.abs(b3[r])))
        assert b3[r, j] > 0
    # negating the data keeps the axes (the convention fixes their signs)
    _, bn, _ = O.pca_fit(-x, 3)
    np.testing.assert_allclose(bn, b3, atol=1e-9)
