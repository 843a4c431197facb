"""Image quality metrics, FP64 (numpy / scipy).

TEST INFRASTRUCTURE ONLY: used by the test suite and the benchmark to check
the library's SSIM / PSNR kernels; never by the product path, and it shares
no code with it.

Section 6 of the paper scores VDI renderings against DVR with SSIM and PSNR
(computed with scikit-image, which is not installed here).  Definitions used:
  - SSIM (Wang, Bovik, Sheikh, Simoncelli 2004): local statistics under an
    11 x 11 Gaussian window with sigma 1.5 (normalised), constants
    C1 = (0.01 L)^2, C2 = (0.03 L)^2 with data range L = 1, population
    (weighted) moments, SSIM map averaged over the pixels whose window lies
    inside the image, then over the R, G, B channels;
  - PSNR = 10 log10(L^2 / MSE), MSE over all pixels and R, G, B.
Images are [H, W, 4] RGBA arrays; the alpha channel is not compared.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

SIGMA = 1.5
RADIUS = 5
K1, K2 = 0.01, 0.03


def gaussian_window(sigma: float = SIGMA, radius: int = RADIUS) -> np.ndarray:
    k = np.arange(-radius, radius + 1, dtype=np.float64)
    g = np.exp(-(k * k) / (2.0 * sigma * sigma))
    g /= g.sum()
    return np.outer(g, g)


def _local_mean(a: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Weighted window mean at every pixel whose window fits inside the image."""
    r = w.shape[0] // 2
    full = ndimage.correlate(a, w, mode="constant", cval=0.0)
    return full[r:-r, r:-r]


def ssim_map(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """SSIM of two single-channel FP64 images at the valid pixels."""
    w = gaussian_window()
    c1, c2 = K1 ** 2, K2 ** 2
    mx, my = _local_mean(x, w), _local_mean(y, w)
    vx = _local_mean(x * x, w) - mx * mx
    vy = _local_mean(y * y, w) - my * my
    cxy = _local_mean(x * y, w) - mx * my
    return ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2))


def ssim(image: np.ndarray, reference: np.ndarray) -> float:
    a = np.asarray(image, dtype=np.float64)
    b = np.asarray(reference, dtype=np.float64)
    if a.shape != b.shape or a.ndim != 3 or a.shape[2] < 3:
        raise ValueError("images must be [H, W, >=3] of the same shape")
    if a.shape[0] < 2 * RADIUS + 1 or a.shape[1] < 2 * RADIUS + 1:
        raise ValueError("images must be at least 11 x 11")
    return float(np.mean([ssim_map(a[..., c], b[..., c]).mean() for c in range(3)]))


def psnr(image: np.ndarray, reference: np.ndarray) -> float:
    a = np.asarray(image, dtype=np.float64)[..., :3]
    b = np.asarray(reference, dtype=np.float64)[..., :3]
    mse = float(np.mean((a - b) ** 2))
    return float("inf") if mse == 0.0 else 10.0 * np.log10(1.0 / mse)
