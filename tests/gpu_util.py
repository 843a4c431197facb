"""Helpers for the GPU parity tests."""
import numpy as np

TOL = 1e-4   # max |dRGBA| of the FP32 HIP path against the FP64 oracle


def sample_pixels(width, height, n, seed=0):
    """n distinct row-major pixel indices, stratified over the image plus the
    four corners and the centre."""
    rng = np.random.default_rng(seed)
    base = rng.choice(width * height, size=min(n, width * height), replace=False)
    extra = [0, width - 1, (height - 1) * width, height * width - 1, (height // 2) * width + width // 2]
    return np.unique(np.concatenate([base, extra]))


def psnr(a, b):
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)
