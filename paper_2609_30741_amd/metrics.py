"""Image-quality measurements for the bench (not part of the frame path).

SSIM follows its published definition (Wang, Bovik, Sheikh and Simoncelli,
2004): per-window luminance, contrast and structure terms from Gaussian-
weighted local means, variances and covariance (an 11x11 window, sigma 1.5,
weights summing to one), C1 = (0.01 L)^2, C2 = (0.03 L)^2 for a data range
L, averaged over the windows that lie wholly inside the image ("valid"
windows), per channel, then over channels.  It is the affiliated-eye
structural-similarity counterpart of the PSNR the paper reports in its
quality table; here it compares the pipeline's affiliated eye with the full
render of that eye.  Computed in fp64 on the host.
"""
from __future__ import annotations

import numpy as np
from scipy.ndimage import gaussian_filter

SSIM_SIGMA = 1.5
SSIM_RADIUS = 5  # an 11x11 window


def _blur(x: np.ndarray) -> np.ndarray:
    # truncate = radius / sigma gives exactly 2 * radius + 1 taps; border
    # handling does not matter for the valid windows kept afterwards.
    return gaussian_filter(x, SSIM_SIGMA, truncate=SSIM_RADIUS / SSIM_SIGMA, mode="reflect")


def ssim_map(x: np.ndarray, y: np.ndarray, data_range: float = 1.0) -> np.ndarray:
    """SSIM of every valid window of two single-channel images [H, W]."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    if x.shape != y.shape or x.ndim != 2:
        raise ValueError("ssim_map takes two images of the same [H, W] shape")
    r = SSIM_RADIUS
    if x.shape[0] <= 2 * r or x.shape[1] <= 2 * r:
        raise ValueError("images must be larger than the 11x11 window")
    c1 = (0.01 * data_range) ** 2
    c2 = (0.03 * data_range) ** 2
    mx, my = _blur(x), _blur(y)
    sxx = _blur(x * x) - mx * mx
    syy = _blur(y * y) - my * my
    sxy = _blur(x * y) - mx * my
    s = ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
    return s[r:-r, r:-r]


def ssim(x: np.ndarray, y: np.ndarray, data_range: float = 1.0) -> float:
    """Mean SSIM of two images, [C, H, W] (channels averaged) or [H, W]."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    if x.ndim == 2:
        return float(ssim_map(x, y, data_range).mean())
    return float(np.mean([ssim_map(x[c], y[c], data_range).mean() for c in range(x.shape[0])]))
