"""FP64 CPU oracle for VDI raycasting.

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the product path.  It shares no
code with the HIP library; both read the same seeded arrays from `inputs`.

Functions (each follows a passage of the paper; see oracle.c for the plain
definitions they implement):
  render_exact      exact raycast of a VDI from a new viewpoint (Sections 4.1-4.2, Eq. 2)
  render_preview    along-ray subsampled preview (Section 4.4) with tie flags
  preview_tie_variants   the preview's valid results where samples rest on ties
  exact_tie_variants     the exact mode's valid results for rays along list edges
  render            full entry point: D_I image downsampling + bilinear upsampling
  count_grid        per-cell supersegment counts (Section 4.3)
  march             brute-force fine-step marching of the same field (a check, not the method)
  dequant_f16 / dequant_bf16   round-to-nearest-even storage of colour (FP16/BF16 forms)
  b_alg             algorithmic bytes of a render, from the touched lists/supersegments
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=gnu11", "-o", tmp, _SRC, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _CVdi(ctypes.Structure):
    _fields_ = [("W", ctypes.c_int32), ("H", ctypes.c_int32), ("NS", ctypes.c_int32),
                ("grid_k", ctypes.c_int32), ("grid_nz", ctypes.c_int32),
                ("cam", ctypes.c_void_p), ("bmin", ctypes.c_void_p), ("bmax", ctypes.c_void_p),
                ("count", ctypes.c_void_p), ("depth", ctypes.c_void_p), ("rgba", ctypes.c_void_p),
                ("grid_z", ctypes.c_void_p), ("grid", ctypes.c_void_p)]


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        I64 = ctypes.c_int64
        lib.or_render_exact.argtypes = [P, P, I, I, ctypes.c_double, I64, P, P, P, P, P, P, P, P, I]
        lib.or_render_preview.argtypes = [P, P, I, I, ctypes.c_double, ctypes.c_double, I64, P, P, P, P, P, I]
        lib.or_upsample.argtypes = [P, P, I, I, I, I, P, P]
        lib.or_upsample.restype = None
        lib.or_count_grid.argtypes = [P, P]
        lib.or_count_grid.restype = None
        lib.or_march.argtypes = [P, P, I, I, I64, P, I64, P, I]
        lib.or_threads.restype = I
        _lib = lib
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


class _Bound:
    """Keeps the arrays a C view points into alive."""

    def __init__(self, vdi, grid: Optional[np.ndarray] = None, rgba: Optional[np.ndarray] = None):
        self.cam = vdi.camera.as_array()
        self.bmin = np.array(vdi.bmin, dtype=np.float64)
        self.bmax = np.array(vdi.bmax, dtype=np.float64)
        self.count = np.ascontiguousarray(vdi.count, dtype=np.uint8)
        self.depth = np.ascontiguousarray(vdi.depth, dtype=np.float32)
        self.rgba = np.ascontiguousarray(vdi.rgba if rgba is None else rgba, dtype=np.float32)
        self.grid_z = np.ascontiguousarray(vdi.grid_z, dtype=np.float32)
        self.grid = None if grid is None else np.ascontiguousarray(grid, dtype=np.uint32)
        self.c = _CVdi(vdi.width, vdi.height, vdi.ns, vdi.grid_k, vdi.grid_nz, _p(self.cam), _p(self.bmin),
                       _p(self.bmax), _p(self.count), _p(self.depth), _p(self.rgba), _p(self.grid_z),
                       _p(self.grid))


def _cam(camera) -> np.ndarray:
    return np.ascontiguousarray(camera.as_array(), dtype=np.float32)


def _pix(pixels) -> Optional[np.ndarray]:
    return None if pixels is None else np.ascontiguousarray(pixels, dtype=np.int64)


def threads() -> int:
    return int(_load().or_threads())


def render_exact(vdi, camera, width: int, height: int, pixels=None, rgba: Optional[np.ndarray] = None,
                 stats: bool = False, touched: bool = False, nthreads: int = 0, aspect: float = 0.0,
                 ess: bool = False, flags: bool = False, bias=None):
    """Exact FP64 render.  Returns out [H, W, 4] (or [npix, 4] for a pixel
    list of row-major indices py*W+px), premultiplied RGB + alpha.
    flags=True returns (out, flags u8) instead: pixels whose ray runs along a
    list edge over part of its length, where either side is a valid reading
    of the field; bias = (bx, by), each -1, 0 or +1, resolves every such tie
    of a ray one way (None: by rounding).
    With stats=True also returns int64 [.., 2] = (lists entered, pieces
    composited), [.., 3] with ess=True (and lists entered over a part of
    the ray inside a non-empty grid cell); with touched=True also
    (touched_lists [H,W] u8, touched_S [NS,H,W] u8) of the VDI, and with
    ess=True also touched_lists_ess [H,W] u8: the lists entered before
    termination over a part of the ray inside a non-empty grid cell (the
    lists empty-space skipping cannot skip, Section 4.3)."""
    lib = _load()
    b = _Bound(vdi, rgba=rgba, grid=count_grid(vdi) if ess else None)
    cam = _cam(camera)
    pix = _pix(pixels)
    n = width * height if pix is None else len(pix)
    out = np.zeros((n, 4), dtype=np.float64)
    st = np.zeros((n, 3), dtype=np.int64) if stats else None
    tl = np.zeros((vdi.height, vdi.width), dtype=np.uint8) if touched else None
    ts = np.zeros((vdi.ns, vdi.height, vdi.width), dtype=np.uint8) if touched else None
    te = np.zeros((vdi.height, vdi.width), dtype=np.uint8) if (touched or stats) and ess else None
    fl = np.zeros(n, dtype=np.uint8) if flags else None
    bb = None if bias is None else np.ascontiguousarray(bias, dtype=np.float64)
    assert bb is None or (bb.shape == (2,) and np.isin(bb, (-1.0, 0.0, 1.0)).all())
    assert not (flags and (stats or touched))
    lib.or_render_exact(ctypes.byref(b.c), _p(cam), width, height, float(aspect), n, _p(pix), _p(out), _p(st),
                        _p(tl), _p(ts), _p(te), _p(fl), _p(bb), nthreads)
    if flags:
        return (out.reshape(height, width, 4), fl.reshape(height, width)) if pix is None else (out, fl)
    if st is not None and not ess:
        st = st[:, :2]
    if pix is None:
        out = out.reshape(height, width, 4)
        if st is not None:
            st = st.reshape(height, width, st.shape[1])
    res = [out]
    if stats:
        res.append(st)
    if touched:
        res.extend([tl, ts])
        if ess:
            res.append(te)
    return res[0] if len(res) == 1 else tuple(res)


def count_grid(vdi) -> np.ndarray:
    """uint32 [grid_nz, ceil(H/k), ceil(W/k)]."""
    k = vdi.grid_k
    gw, gh = -(-vdi.width // k), -(-vdi.height // k)
    out = np.zeros((vdi.grid_nz, gh, gw), dtype=np.uint32)
    b = _Bound(vdi)
    _load().or_count_grid(ctypes.byref(b.c), _p(out))
    return out


def lowres_size(width: int, height: int, d_i: float):
    """Image size rendered for downsampling factor D_I >= 1 (round half up, >= 1)."""
    return max(1, int(np.floor(width / d_i + 0.5))), max(1, int(np.floor(height / d_i + 0.5)))


def render_preview(vdi, camera, w: int, h: int, d_r: float, pixels=None, grid: Optional[np.ndarray] = None,
                   rgba: Optional[np.ndarray] = None, nthreads: int = 0, samples: bool = False, aspect: float = 0.0,
                   bias=None):
    """Along-ray subsampled render of a w x h image (D_R > 0); aspect 0
    means w/h.  Returns (out [h, w, 4], flags [h, w] u8) or per-pixel arrays
    for a pixel list.  bias = (bx, by, bz, bn), each -1, 0 or +1, resolves
    every tie of a ray one way (list edges in x and y, supersegment faces,
    sample-count thresholds); None leaves ties to rounding."""
    lib = _load()
    if grid is None:
        grid = count_grid(vdi)
    b = _Bound(vdi, grid=grid, rgba=rgba)
    cam = _cam(camera)
    pix = _pix(pixels)
    n = w * h if pix is None else len(pix)
    out = np.zeros((n, 4), dtype=np.float64)
    flags = np.zeros(n, dtype=np.uint8)
    ns = np.zeros(n, dtype=np.int64)
    bb = None if bias is None else np.ascontiguousarray(bias, dtype=np.float64)
    assert bb is None or (bb.shape == (4,) and np.isin(bb, (-1.0, 0.0, 1.0)).all())
    rc = lib.or_render_preview(ctypes.byref(b.c), _p(cam), w, h, float(aspect), float(d_r), n, _p(pix), _p(out),
                               _p(flags), _p(ns), _p(bb), nthreads)
    if rc != 0:
        raise ValueError("render_preview needs D_R > 0")
    if pix is None:
        out, flags, ns = out.reshape(h, w, 4), flags.reshape(h, w), ns.reshape(h, w)
    return (out, flags, ns) if samples else (out, flags)


TIE_BIASES = [(bx, by, bz, bn) for bx in (-1, 1) for by in (-1, 1) for bz in (-1, 1) for bn in (-1, 1)]


def preview_tie_variants(vdi, camera, w: int, h: int, d_r: float, pixels, grid: Optional[np.ndarray] = None,
                         rgba: Optional[np.ndarray] = None, nthreads: int = 0, aspect: float = 0.0) -> np.ndarray:
    """The valid results of flagged preview pixels (Section 4.4 sampling
    rule): the pixels rendered once per way of resolving their ties
    consistently along the ray (TIE_BIASES, 16 ways).  Returns
    [len(TIE_BIASES), npix, 4]; a result that rests on ties is correct when
    it equals one of these."""
    if grid is None:
        grid = count_grid(vdi)
    return np.stack([render_preview(vdi, camera, w, h, d_r, pixels=pixels, grid=grid, rgba=rgba, nthreads=nthreads,
                                    aspect=aspect, bias=b)[0] for b in TIE_BIASES])


EXACT_TIE_BIASES = [(bx, by) for bx in (-1, 1) for by in (-1, 1)]


def exact_tie_variants(vdi, camera, w: int, h: int, pixels, rgba: Optional[np.ndarray] = None, nthreads: int = 0,
                       aspect: float = 0.0) -> np.ndarray:
    """The valid exact results of pixels whose rays run along list edges:
    rendered once per way of resolving those ties consistently along the ray
    (EXACT_TIE_BIASES, 4 ways).  Returns [4, npix, 4]."""
    return np.stack([render_exact(vdi, camera, w, h, pixels=pixels, rgba=rgba, nthreads=nthreads, aspect=aspect,
                                  flags=True, bias=b)[0] for b in EXACT_TIE_BIASES])


def upsample(lo: np.ndarray, width: int, height: int, lo_flags: Optional[np.ndarray] = None):
    """Bilinear upsampling (half-pixel centres, clamped) of lo [h, w, 4]."""
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    h, w = lo.shape[:2]
    out = np.zeros((height, width, 4), dtype=np.float64)
    fl = np.zeros((height, width), dtype=np.uint8)
    lf = None if lo_flags is None else np.ascontiguousarray(lo_flags, dtype=np.uint8)
    _load().or_upsample(_p(lo), _p(lf), w, h, width, height, _p(out), _p(fl))
    return out, fl


def render(vdi, camera, width: int, height: int, d_i: float = 1.0, d_r: float = 0.0,
           rgba: Optional[np.ndarray] = None, nthreads: int = 0):
    """The full render: exact (D_R = 0) or along-ray subsampled (D_R > 0) at
    round(W/D_I) x round(H/D_I) with the display's aspect W/H, then bilinear
    upsampling to W x H when D_I > 1 (Section 4.4).
    Returns (out [H, W, 4] float64, flags [H, W] uint8)."""
    w, h = lowres_size(width, height, d_i)
    aspect = width / height
    if d_r > 0.0:
        lo, fl = render_preview(vdi, camera, w, h, d_r, rgba=rgba, nthreads=nthreads, aspect=aspect)
    else:
        lo, fl = render_exact(vdi, camera, w, h, rgba=rgba, nthreads=nthreads, aspect=aspect, flags=True)
    if (w, h) == (width, height):
        return lo, fl
    return upsample(lo, width, height, fl)


def march(vdi, camera, width: int, height: int, pixels, steps: int, nthreads: int = 0) -> np.ndarray:
    lib = _load()
    b = _Bound(vdi)
    cam = _cam(camera)
    pix = _pix(pixels)
    out = np.zeros((len(pix), 4), dtype=np.float64)
    lib.or_march(ctypes.byref(b.c), _p(cam), width, height, len(pix), _p(pix), int(steps), _p(out), nthreads)
    return out


# ----------------------------------------------------------------------------
# Storage precision forms (round to nearest, ties to even)
# ----------------------------------------------------------------------------
def dequant_f16(x: np.ndarray) -> np.ndarray:
    """float32 -> IEEE binary16 (round to nearest even, numpy's conversion) -> float32."""
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float32)


def dequant_bf16(x: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 by rounding the low 16 bits to nearest, ties to
    even (finite inputs; the largest finite values round to infinity as IEEE
    rounding does), -> float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    lsb = (u >> np.uint32(16)) & np.uint32(1)
    r = (u + np.uint32(0x7FFF) + lsb) & np.uint32(0xFFFF0000)
    return r.view(np.float32)


# ----------------------------------------------------------------------------
# Algorithmic bytes
# ----------------------------------------------------------------------------
def b_alg(vdi, touched_lists: np.ndarray, touched_s: np.ndarray, out_pixels: int, colour_bytes: int = 16) -> int:
    """Bytes the method must move for one render: per list entered by a ray
    before its termination, its count byte and all its (f, b) pairs; per
    supersegment composited, its colour; plus the RGBA32F output."""
    n = vdi.count.astype(np.int64)
    lists = touched_lists.astype(bool)
    return int(lists.sum() + 8 * n[lists].sum() + colour_bytes * int(touched_s.astype(bool).sum()) + 16 * out_pixels)


def render_points(vdi, camera, width: int, height: int, d_i: float, d_r: float, pixels,
                  rgba: Optional[np.ndarray] = None, nthreads: int = 0):
    """Selected output pixels (row-major indices) of `render`: the low-res
    texels each one's bilinear filter reads are rendered one by one and
    combined with the same weights as `upsample`.  Returns (values [n, 4],
    flags [n])."""
    pixels = np.asarray(pixels, dtype=np.int64)
    w, h = lowres_size(width, height, d_i)
    aspect = width / height

    def lo_render(pix):
        if d_r > 0.0:
            return render_preview(vdi, camera, w, h, d_r, pixels=pix, rgba=rgba, nthreads=nthreads, aspect=aspect)
        return render_exact(vdi, camera, w, h, pixels=pix, rgba=rgba, nthreads=nthreads, aspect=aspect, flags=True)

    if (w, h) == (width, height):
        return lo_render(pixels)
    x, y = pixels % width, pixels // width
    sx = np.clip((x + 0.5) * w / width - 0.5, 0.0, w - 1)
    sy = np.clip((y + 0.5) * h / height - 0.5, 0.0, h - 1)
    x0, y0 = np.floor(sx).astype(np.int64), np.floor(sy).astype(np.int64)
    x1, y1 = np.minimum(x0 + 1, w - 1), np.minimum(y0 + 1, h - 1)
    fx, fy = sx - x0, sy - y0
    taps = [y0 * w + x0, y0 * w + x1, y1 * w + x0, y1 * w + x1]
    need, inv = np.unique(np.concatenate(taps), return_inverse=True)
    vals, fl = lo_render(need)
    n = len(pixels)
    a, b, c, d = (vals[inv[k * n:(k + 1) * n]] for k in range(4))
    out = (a * (1 - fx)[:, None] + b * fx[:, None]) * (1 - fy)[:, None] + \
          (c * (1 - fx)[:, None] + d * fx[:, None]) * fy[:, None]
    flags = np.zeros(n, np.uint8)
    for k in range(4):
        flags |= fl[inv[k * n:(k + 1) * n]]
    return out, flags
