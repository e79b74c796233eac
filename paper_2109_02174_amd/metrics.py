"""Image agreement metrics: max-abs and RMSE normalised by a value range, PSNR, SSIM.

PSNR follows Eq. 3 of arXiv 2109.02174 (section "Benchmark"):
PSNR = 20 log10(MAX / sqrt(MSE)), infinite for identical images.  The paper
leaves MAX undefined; here MAX is the phantom range R (max - min of the
pixel-centre raster).  SSIM follows Eq. 4 with the constants and 11x11
Gaussian window (sigma 1.5) of Wang et al. 2004, which the paper does not
state.
"""
from __future__ import annotations

import math

import numpy as np


def max_abs(a, b) -> float:
    return float(np.max(np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64))))


def rmse(a, b) -> float:
    d = np.asarray(a, np.float64) - np.asarray(b, np.float64)
    return float(math.sqrt(np.mean(d * d))) if d.size else 0.0


def psnr(a, b, max_value: float) -> float:
    """20 log10(max_value / RMSE); +inf when the images are identical."""
    e = rmse(a, b)
    if e == 0.0:
        return math.inf
    return 20.0 * math.log10(max_value / e)


def compare(test, ref, value_range: float) -> dict:
    """max-abs/R, RMSE/R and PSNR(MAX = R) of ``test`` against ``ref``."""
    R = float(value_range)
    return {"max_abs_rel": max_abs(test, ref) / R, "rmse_rel": rmse(test, ref) / R,
            "psnr_db": psnr(test, ref, R)}


def _gauss_window(size: int = 11, sigma: float = 1.5) -> np.ndarray:
    ax = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-ax * ax / (2.0 * sigma * sigma))
    g /= g.sum()
    return g


def _filter2(img: np.ndarray, g: np.ndarray) -> np.ndarray:
    """'valid' separable 2D correlation with the 1D window g."""
    from numpy.lib.stride_tricks import sliding_window_view
    rows = sliding_window_view(img, g.size, axis=1) @ g
    return sliding_window_view(rows, g.size, axis=0) @ g


def ssim(a, b, value_range: float, k1: float = 0.01, k2: float = 0.03) -> float:
    """Mean SSIM (Eq. 4) over 11x11 Gaussian windows."""
    x = np.asarray(a, np.float64)
    y = np.asarray(b, np.float64)
    g = _gauss_window()
    c1 = (k1 * value_range) ** 2
    c2 = (k2 * value_range) ** 2
    mx, my = _filter2(x, g), _filter2(y, g)
    sxx = _filter2(x * x, g) - mx * mx
    syy = _filter2(y * y, g) - my * my
    sxy = _filter2(x * y, g) - mx * my
    s = ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
    return float(np.mean(s))
