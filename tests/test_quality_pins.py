"""Pins of the quality oracle (SSIM / PSNR, Section 6) and of the CPU
generator's DVR image, the reference the GPU DVR and the quality sweep are
checked against.  Every expected value here comes from a closed form, a
textbook property or a brute-force loop, not from the code under test."""
import math

import numpy as np
import pytest

import inputs
from oracle import quality as Q


def _rgba(rgb):
    a = np.ones(rgb.shape[:2] + (1,))
    return np.concatenate([rgb, a], axis=2)


def test_ssim_identity_symmetry_and_range():
    rng = np.random.default_rng(5)
    x = _rgba(rng.random((24, 31, 3)))
    y = _rgba(np.clip(x[..., :3] + 0.1 * rng.standard_normal((24, 31, 3)), 0, 1))
    assert Q.ssim(x, x) == pytest.approx(1.0, abs=1e-12)
    assert Q.ssim(x, y) == pytest.approx(Q.ssim(y, x), abs=1e-14)
    assert -1.0 <= Q.ssim(x, y) < 1.0
    with pytest.raises(ValueError):
        Q.ssim(x[:10], x[:10])


def test_ssim_constant_images_closed_form():
    # Zero variance: the structure term is C2/C2 = 1 and SSIM = (2ab + C1) / (a^2 + b^2 + C1).
    c1 = 0.01 ** 2
    for a, b in [(0.2, 0.2), (0.2, 0.7), (0.0, 1.0), (0.5, 0.45)]:
        x = _rgba(np.full((16, 20, 3), a))
        y = _rgba(np.full((16, 20, 3), b))
        assert Q.ssim(x, y) == pytest.approx((2 * a * b + c1) / (a * a + b * b + c1), abs=1e-12)


def test_ssim_brute_force_tiny():
    # Direct loops over every valid pixel and its 11 x 11 window.
    rng = np.random.default_rng(9)
    x = rng.random((13, 15, 3))
    y = np.clip(x + 0.2 * rng.standard_normal(x.shape), 0, 1)
    g = [math.exp(-(k * k) / (2 * 1.5 * 1.5)) for k in range(-5, 6)]
    sg = sum(g)
    g = [v / sg for v in g]
    tot = 0.0
    n = 0
    for c in range(3):
        for i in range(5, 13 - 5):
            for j in range(5, 15 - 5):
                mx = my = sxx = syy = sxy = 0.0
                for di in range(-5, 6):
                    for dj in range(-5, 6):
                        w = g[di + 5] * g[dj + 5]
                        a, b = x[i + di, j + dj, c], y[i + di, j + dj, c]
                        mx += w * a
                        my += w * b
                        sxx += w * a * a
                        syy += w * b * b
                        sxy += w * a * b
                vx, vy, cv = sxx - mx * mx, syy - my * my, sxy - mx * my
                tot += ((2 * mx * my + 1e-4) * (2 * cv + 9e-4)) / ((mx * mx + my * my + 1e-4) * (vx + vy + 9e-4))
                n += 1
    assert Q.ssim(_rgba(x), _rgba(y)) == pytest.approx(tot / n, abs=1e-12)


def test_psnr_closed_form():
    rng = np.random.default_rng(2)
    x = _rgba(rng.random((20, 20, 3)) * 0.5)
    for c in (0.1, 0.01, 0.001):
        y = x.copy()
        y[..., :3] += c
        y[..., 3] = 0.0   # alpha is not compared
        assert Q.psnr(y, x) == pytest.approx(-20 * math.log10(c), abs=1e-9)
    assert Q.psnr(x, x) == float("inf")


# --- The CPU generator's DVR image (the emission-absorption integral of Section 2) ---

def _ray_box_length(eye, d, lo=-0.5, hi=0.5):
    """Textbook slab test: length of the ray inside the cube [lo, hi]^3."""
    t0, t1 = -math.inf, math.inf
    for a in range(3):
        if abs(d[a]) < 1e-300:
            continue
        ta, tb = (lo - eye[a]) / d[a], (hi - eye[a]) / d[a]
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    return max(0.0, t1 - t0)


def test_generator_dvr_of_constant_volume_is_beer_lambert():
    # A constant field v: every sample has the same colour c and opacity a_tf,
    # a sample of length len has opacity 1 - (1 - a_tf)^(len/ds), so the ray's
    # transmittance is (1 - a_tf)^(L/ds) for its length L in the cube, and its
    # colour c (1 - T).  Ramp TF: c = (v, 0.25 + 0.5 v, 1 - v), a_tf = 0.2 (v - 0.05)/0.95.
    n, v = 32, 0.3
    vol = np.full((n, n, n), v, np.float32)
    W, H = 9, 7
    cam = inputs.orbit_camera(0.0)
    out = inputs.generate_vdi(vol, cam, W, H, 1, inputs.TF_RAMP, gamma=1.0)
    vv = float(np.float32(v))
    atf = 0.2 * (vv - 0.05) / 0.95
    ds = 1.0 / n
    th = math.tan(math.radians(inputs.FOV_Y_DEG) / 2)
    eye = (0.0, 0.0, float(np.float32(inputs.ORBIT_RADIUS)))
    for py in range(H):
        for px in range(W):
            xc, yc = -1 + (2 * px + 1) / W, -1 + (2 * py + 1) / H
            d = np.array([xc * th * W / H, yc * th, -1.0])
            d /= np.linalg.norm(d)
            L = _ray_box_length(eye, d)
            T = (1 - atf) ** (L / ds)
            want = [vv * (1 - T), (0.25 + 0.5 * vv) * (1 - T), (1 - vv) * (1 - T), 1 - T]
            assert np.allclose(out.dvr[py, px], want, atol=1e-12, rtol=1e-12), (px, py, out.dvr[py, px], want)


def test_generator_dvr_early_termination_and_empty_volume():
    n = 128
    vol = np.ones((n, n, n), np.float32)          # knots TF: opacity 0.12 per voxel length
    out = inputs.generate_vdi(vol, inputs.orbit_camera(0.0), 8, 8, 1, inputs.TF_KNOTS4, gamma=1.0)
    # The central rays cross ~128 voxels: 0.88^128 < 1e-7 without termination.
    a = out.dvr[2:6, 2:6, 3]
    # Marching stops at the first sample that takes the transmittance to <= 1e-5;
    # a sample is at most one voxel long, so it removes at most 12% of it.
    assert (1 - a <= 1e-5).all() and (1 - a > 1e-5 * (1 - 0.12)).all()
    assert np.allclose(out.dvr[2:6, 2:6, :3], np.array([0.9, 0.15, 0.1]) * a[..., None], rtol=1e-12, atol=0)
    empty = inputs.generate_vdi(np.zeros((8, 8, 8), np.float32), inputs.orbit_camera(10.0), 8, 8, 1,
                                inputs.TF_RAMP, gamma=1.0)
    assert not empty.dvr.any()
