"""The bench's SSIM against its definition: closed forms and an explicit
window sum."""
import math

import numpy as np
import pytest

from paper_2609_30741_amd import metrics


def test_identical_images_give_one():
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 1, size=(3, 40, 52))
    assert metrics.ssim(x, x) == pytest.approx(1.0, abs=1e-12)


def test_constant_images_closed_form():
    # No variance anywhere: the contrast-structure term is C2 / C2 = 1 and
    # every window's luminance term is (2ab + C1) / (a^2 + b^2 + C1).
    a, b = 0.3, 0.7
    c1 = (0.01) ** 2
    x = np.full((30, 30), a)
    y = np.full((30, 30), b)
    assert metrics.ssim(x, y) == pytest.approx((2 * a * b + c1) / (a * a + b * b + c1), rel=1e-12)


def test_constant_offset_keeps_structure():
    # y = x + c: equal variances and covariance, so only the luminance term
    # of each window's local mean m remains, (2 m (m + c) + C1) / (m^2 + (m + c)^2 + C1).
    rng = np.random.default_rng(1)
    x = rng.uniform(0.2, 0.6, size=(32, 28))
    c = 0.15
    m = metrics._blur(x)[5:-5, 5:-5]
    c1 = (0.01) ** 2
    want = (2 * m * (m + c) + c1) / (m * m + (m + c) ** 2 + c1)
    np.testing.assert_allclose(metrics.ssim_map(x, x + c), want, rtol=1e-9)


def test_window_matches_an_explicit_gaussian_sum():
    # One valid window summed by hand: 11x11 Gaussian weights of sigma 1.5,
    # normalised to one, local means, variances and covariance.
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, size=(24, 30))
    y = np.clip(x + rng.normal(0, 0.1, size=x.shape), 0, 1)
    p, q = 11, 17
    num = np.zeros((11, 11))
    for i in range(-5, 6):
        for j in range(-5, 6):
            num[i + 5, j + 5] = math.exp(-(i * i + j * j) / (2 * 1.5 ** 2))
    w = num / num.sum()
    wx = x[p - 5:p + 6, q - 5:q + 6]
    wy = y[p - 5:p + 6, q - 5:q + 6]
    mx, my = (w * wx).sum(), (w * wy).sum()
    vx = (w * (wx - mx) ** 2).sum()
    vy = (w * (wy - my) ** 2).sum()
    cxy = (w * (wx - mx) * (wy - my)).sum()
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    want = (2 * mx * my + c1) * (2 * cxy + c2) / ((mx * mx + my * my + c1) * (vx + vy + c2))
    got = metrics.ssim_map(x, y)[p - 5, q - 5]
    assert got == pytest.approx(want, rel=1e-9)


def test_symmetric_and_below_one_for_different_images():
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, size=(3, 25, 25))
    y = np.clip(x + rng.normal(0, 0.2, size=x.shape), 0, 1)
    s = metrics.ssim(x, y)
    assert s == pytest.approx(metrics.ssim(y, x), rel=1e-12)
    assert 0.0 < s < 0.99


def test_rejects_images_no_larger_than_the_window():
    with pytest.raises(ValueError):
        metrics.ssim(np.zeros((10, 40)), np.zeros((10, 40)))
