"""Helpers for the GPU parity tests."""
import numpy as np

TOL = 1e-4   # max |dRGBA| of the FP32 HIP path against the FP64 oracle


def sample_pixels(width, height, n, seed=0):
    """About n distinct row-major pixel indices: half uniform over the image,
    half over its central region (where the volumes project), plus the four
    corners and the centre."""
    rng = np.random.default_rng(seed)
    uni = rng.choice(width * height, size=min(n // 2, width * height), replace=False)
    cx = rng.integers(width // 4, max(width // 4 + 1, 3 * width // 4), size=n - n // 2)
    cy = rng.integers(height // 8, max(height // 8 + 1, 7 * height // 8), size=n - n // 2)
    extra = [0, width - 1, (height - 1) * width, height * width - 1, (height // 2) * width + width // 2]
    return np.unique(np.concatenate([uni, cy * width + cx, extra]))


def psnr(a, b):
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)
