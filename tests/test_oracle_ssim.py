"""Pins of the oracle's SSIM term (CPU): identity and symmetry, closed forms
that fix C1 and C2 separately, the window sums against scipy's Gaussian
filter (an independent library routine), and the gradient against central
finite differences."""
import numpy as np
import pytest

from oracle import ssim as S

scipy_ndimage = pytest.importorskip("scipy.ndimage")
# the definition's constants (Wang et al. 2004: C = (K L)^2, K1 = 0.01, K2 = 0.03,
# dynamic range L = 1), written here rather than read from the oracle
C1, C2 = 0.01 ** 2, 0.03 ** 2


def imgs(seed, shape=(2, 3, 9, 13)):
    rng = np.random.default_rng(seed)
    return rng.random(shape), rng.random(shape)


def test_identity_and_symmetry():
    x, y = imgs(0)
    assert abs(S.ssim(x, x) - 1.0) < 1e-15
    assert abs(S.ssim(x, y) - S.ssim(y, x)) < 1e-15
    assert S.ssim(x, y) < 0.9


def test_window_sums_match_scipy_gaussian_filter():
    """11 taps of sigma 1.5 normalised = scipy's filter with radius 5; zero
    outside the image = mode 'constant'."""
    x, _ = imgs(1, (17, 23))
    ref = scipy_ndimage.gaussian_filter(x, 1.5, truncate=5 / 1.5, mode="constant", cval=0.0)
    assert np.allclose(S.filt(x), ref, rtol=0, atol=1e-14)
    g = S.window()
    assert g.size == 11 and abs(g.sum() - 1) < 1e-15 and np.allclose(g, g[::-1])


def test_constant_images_fix_c1():
    """Interior pixels of constant images a, b: zero variances, S reduces to
    (2ab + C1) / (a^2 + b^2 + C1)."""
    a, b = 0.3, 0.7
    x = np.full((20, 20), a)
    y = np.full((20, 20), b)
    m = S.ssim_map(x, y)[6:-6, 6:-6]
    assert np.allclose(m, (2 * a * b + C1) / (a * a + b * b + C1), rtol=1e-12)


def test_mirrored_image_fixes_c2():
    """y = 1 - x: equal means are not needed; the covariance is minus the
    variance, so S = L (C2 - 2v) / (C2 + 2v) with L the luminance term and v
    the window variance of x, computed here as the weighted mean of squared
    deviations (two passes, not the moment formula)."""
    rng = np.random.default_rng(3)
    x = rng.random((25, 25))
    y = 1.0 - x
    g = S.window()
    w2 = np.outer(g, g)
    m = S.ssim_map(x, y)
    for (i, j) in [(12, 12), (7, 15), (18, 9)]:
        patch = x[i - 5:i + 6, j - 5:j + 6]
        mu = (w2 * patch).sum()
        v = (w2 * (patch - mu) ** 2).sum()
        muy = 1.0 - mu
        L = (2 * mu * muy + C1) / (mu * mu + muy * muy + C1)
        assert abs(m[i, j] - L * (C2 - 2 * v) / (C2 + 2 * v)) < 1e-12


def test_gradient_against_finite_differences():
    x, y = imgs(4, (1, 2, 8, 11))
    g = S.ssim_grad(x, y)
    rng = np.random.default_rng(5)
    h = 1e-6
    for idx in [tuple(rng.integers(0, d) for d in x.shape) for _ in range(25)] + \
               [(0, 0, 0, 0), (0, 1, 7, 10), (0, 0, 3, 0)]:
        xp = x.copy()
        xm = x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (S.ssim(xp, y) - S.ssim(xm, y)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-7 * max(abs(g).max(), 1e-12), (idx, fd, g[idx])
    loss, dl = S.dssim_loss(x, y, 0.2)
    assert abs(loss - 0.2 * (1 - S.ssim(x, y))) < 1e-15 and np.allclose(dl, -0.2 * g)
