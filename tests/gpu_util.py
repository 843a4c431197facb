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


def tie_aware_errors(img, ref, flags, variants):
    """Per-pixel error of preview pixels: |img - ref| (max over RGBA) where
    the oracle's result is unique (flags == 0); where it rests on ties, the
    distance to the nearest of the valid results `variants`
    [n_variants, n_flagged, 4] (oracle.preview_tie_variants of the flagged
    pixels, in order).  Returns (errors [n], index of the nearest variant
    per flagged pixel)."""
    img = np.asarray(img, np.float64)
    err = np.abs(img - ref).max(axis=1)
    fl = np.flatnonzero(flags != 0)
    if len(fl) == 0:
        return err, np.zeros(0, np.int64)
    d = np.abs(np.asarray(variants)[:, :, :] - img[fl][None]).max(axis=2)
    err[fl] = d.min(axis=0)
    return err, d.argmin(axis=0)


def preview_errors(img_px, src, cam, w, h, d_r, pix, aspect=0.0, grid=None, rgba=None):
    """Errors of a w x h along-ray subsampled render (D_I = 1 on that grid)
    at pixel list `pix` (img_px [n, 4]) against the oracle, ties included:
    unflagged pixels against the unique result, flagged ones against the
    nearest consistent tie resolution.  Returns (errors [n], flags [n],
    oracle values [n, 4])."""
    import oracle
    pix = np.asarray(pix, np.int64)
    ref, flags = oracle.render_preview(src, cam, w, h, d_r, pixels=pix, aspect=aspect, grid=grid, rgba=rgba)
    var = None
    if flags.any():
        var = oracle.preview_tie_variants(src, cam, w, h, d_r, pix[flags != 0], aspect=aspect, grid=grid, rgba=rgba)
    err, _ = tie_aware_errors(img_px, ref, flags, var)
    return err, flags, ref


def exact_errors(img_px, src, cam, w, h, pix, aspect=0.0, rgba=None):
    """Errors of an exact w x h render at pixel list `pix` (img_px [n, 4])
    against the oracle: rays off list edges against the unique result, rays
    running along a list edge (oracle flag) against the nearest of its four
    consistent tie resolutions.  Returns (errors [n], flags [n], oracle
    values [n, 4])."""
    import oracle
    pix = np.asarray(pix, np.int64)
    ref, flags = oracle.render_exact(src, cam, w, h, pixels=pix, aspect=aspect, rgba=rgba, flags=True)
    var = None
    if flags.any():
        var = oracle.exact_tie_variants(src, cam, w, h, pix[flags != 0], aspect=aspect, rgba=rgba)
    err, _ = tie_aware_errors(img_px, ref, flags, var)
    return err, flags, ref


def nonempty_stratum(img, n, seed=0):
    """Up to n row-major indices of pixels with positive alpha in img [H, W, 4]
    (picks where to look; the expected values come from the oracle)."""
    idx = np.flatnonzero(np.asarray(img)[..., 3].reshape(-1) > 0)
    if len(idx) <= n:
        return idx
    return np.random.default_rng(seed).choice(idx, n, replace=False)


def oracle_check(src, rgba, cam, W, H, d_i, d_r, img, n=1500, seed=0, min_ok=0.9):
    """A rendered image against the oracle on sampled pixels (a stratum of them
    non-empty).  Exact frames and D_I = 1 previews pixel by pixel (preview
    ties against every consistent resolution); downsampled previews on the
    pixels whose four low-res texels rest on no tie (at least a fraction
    min_ok of the sample).  Returns the number of non-empty pixels compared."""
    img = img.reshape(-1, 4).astype(np.float64)
    pix = np.unique(np.concatenate([sample_pixels(W, H, n, seed=seed),
                                    nonempty_stratum(img.reshape(H, W, 4), n // 2, seed=seed)]))
    if d_r > 0 and d_i == 1.0:
        err, _, ref = preview_errors(img[pix], src, cam, W, H, d_r, pix, rgba=rgba)
        ok = np.ones(len(pix), bool)
    else:
        import oracle
        ref, flags = oracle.render_points(src, cam, W, H, d_i, d_r, pix, rgba=rgba)
        ok = flags == 0
        err = np.abs(img[pix] - ref).max(axis=1)
    assert ok.mean() > min_ok, float(ok.mean())
    assert err[ok].max() <= TOL, (d_i, d_r, float(err[ok].max()))
    return int((ok & (ref[:, 3] > 0)).sum())
