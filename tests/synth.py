"""Hand-built VDIs with known answers, used by the oracle pins and the GPU
parity tests.  Plain data construction; no rendering arithmetic."""
from __future__ import annotations

import math

import numpy as np

import inputs


def empty_vdi(w: int, h: int, ns: int, camera=None, half: float = 0.5, box=None) -> inputs.VDI:
    cam = camera or inputs.orbit_camera(0.0)
    bmin, bmax = box if box is not None else ((-half,) * 3, (half,) * 3)
    return inputs.VDI(width=w, height=h, ns=ns, camera=cam, bmin=bmin, bmax=bmax,
                      count=np.zeros((h, w), np.uint8), depth=np.zeros((ns, h, w, 2), np.float32),
                      rgba=np.zeros((ns, h, w, 4), np.float32))


def list_cos(camera, w: int, h: int) -> np.ndarray:
    """cos of the angle between each list's generating ray and the view axis,
    from the pinhole model (independent of the renderers' code)."""
    th = math.tan(math.radians(camera.fov_y_deg) / 2.0)
    xs = -1.0 + (2.0 * np.arange(w) + 1.0) / w
    ys = -1.0 + (2.0 * np.arange(h) + 1.0) / h
    X, Y = np.meshgrid(xs * th * w / h, ys * th)
    return 1.0 / np.sqrt(1.0 + X * X + Y * Y)


def slab_vdi(w: int, h: int, slabs, ns: int = None, half: float = 4.0) -> inputs.VDI:
    """Homogeneous slabs between planes of constant V_O view depth.
    slabs = [(z1, z2, sigma, (r, g, b)), ...] front to back.  Every list gets
    one supersegment per slab with opacity 1 - exp(-sigma (z2-z1)/cos_i), so a
    ray crossing slab s with world length L sees opacity 1 - exp(-sigma L)."""
    ns = ns or len(slabs)
    v = empty_vdi(w, h, ns, half=half)
    cs = list_cos(v.camera, w, h)
    for j, (z1, z2, sig, col) in enumerate(slabs):
        v.depth[j, ..., 0] = z1
        v.depth[j, ..., 1] = z2
        v.rgba[j, ..., 0:3] = col
        v.rgba[j, ..., 3] = (1.0 - np.exp(-sig * (np.float32(z2) - np.float64(np.float32(z1))) / cs)).astype(np.float32)
    v.count[:] = len(slabs)
    v.grid_z = inputs.grid_z_for(v.camera, v.bmin, v.bmax, v.grid_nz)
    return v


def random_vdi(w: int, h: int, ns: int, seed: int, zlo: float = 1.0, zhi: float = 2.0, empty_frac: float = 0.2,
               alpha_max: float = 0.9, min_thick: float = 0.0) -> inputs.VDI:
    """Random valid VDI: per list a random count, sorted non-overlapping
    [f, b] intervals inside [zlo, zhi] (each at least min_thick deep), random
    straight colours and opacities.  The AABB is the smallest box around the
    V_O frustum between depths zlo and zhi (V_O looks down -z from z = 1.5),
    so it encloses every supersegment."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cam = inputs.orbit_camera(0.0)
    th = math.tan(math.radians(cam.fov_y_deg) / 2.0)
    hx, hy = 1.01 * zhi * th * w / h, 1.01 * zhi * th
    ez = cam.eye[2]
    box = ((-hx, -hy, ez - zhi - 1e-3), (hx, hy, ez - zlo + 1e-3))
    v = empty_vdi(w, h, ns, camera=cam, box=box)
    cnt = rng.integers(0, ns + 1, size=(h, w))
    cnt[rng.random((h, w)) < empty_frac] = 0
    for py in range(h):
        for px in range(w):
            n = int(cnt[py, px])
            if n == 0:
                continue
            edges = np.sort(rng.uniform(zlo, zhi, size=2 * n)).astype(np.float32)
            f, b = edges[0::2], edges[1::2]
            ok = b > f + min_thick
            f, b = f[ok], b[ok]
            n = len(f)
            v.count[py, px] = n
            v.depth[:n, py, px, 0] = f
            v.depth[:n, py, px, 1] = b
            v.rgba[:n, py, px, :3] = rng.random((n, 3))
            v.rgba[:n, py, px, 3] = rng.uniform(0.0, alpha_max, size=n)
    v.grid_z = inputs.grid_z_for(v.camera, v.bmin, v.bmax, v.grid_nz)
    return v


def composite_at_vo(v: inputs.VDI, t_term: float = 1e-5) -> np.ndarray:
    """Front-to-back composite of each list's own supersegments (what the
    generating ray accumulated), with termination at transmittance t_term."""
    H, W = v.count.shape
    out = np.zeros((H, W, 4))
    T = np.ones((H, W))
    live = np.ones((H, W), bool)
    for j in range(v.ns):
        a = v.rgba[j, ..., 3].astype(np.float64) * ((v.count > j) & live)
        out[..., :3] += (T * a)[..., None] * v.rgba[j, ..., :3]
        T = T * (1.0 - a)
        live &= T > t_term
    out[..., 3] = 1.0 - T
    return out


def mirror_x(v: inputs.VDI) -> inputs.VDI:
    """VDI made symmetric under x -> -x by copying its left half onto its right."""
    w = v.width
    for arr in (v.count, ):
        arr[:, w - w // 2:] = arr[:, :w // 2][:, ::-1]
    v.depth[:, :, w - w // 2:] = v.depth[:, :, :w // 2][:, :, ::-1]
    v.rgba[:, :, w - w // 2:] = v.rgba[:, :, :w // 2][:, :, ::-1]
    return v
