"""Seeded synthetic inputs for the VDI renderer.

This module is the one place both sides of every comparison get their inputs
from: seeded volumes, transfer functions, the VDI generated from them (the
paper's Section 3: homogeneity criterion of Eq. 1, per-ray sensitivity by the
bisection of supplement Algorithm S1), cameras and the ESS grid's depth-slice
boundaries.  It holds none of the renderer's arithmetic; the FP64 oracle and
the HIP library each consume the arrays it produces and share nothing else.

Workloads (the paper's datasets, Table 1, are not available; these seeded
volumes stand in for them):
  1  tiny     64^3 f32 Gaussian blobs, ramp TF, VDI 128x128, N_S=16, fixed gamma 0.05
  2  720p     512^3 u16 mixing-layer slab of fractal value noise, 4-knot TF,
              VDI 1280x720, N_S=20, per-ray gamma bisection
  3  1080p    1024x1024x512 f32 turbulence in a thresholded shell, 4-knot TF,
              VDI 1920x1080, N_S=50, per-ray gamma bisection
Seeds: volume seed = 1000 + workload number; blob parameters from numpy PCG64.
"""
from __future__ import annotations

import ctypes
import dataclasses
import hashlib
import json
import math
import os
import subprocess
import sys
import time
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_REPO = os.path.dirname(_HERE)
_SRC = os.path.join(_HERE, "vdigen.c")
_LIB = os.path.join(_HERE, "libvdigen.so")
GENERATOR_VERSION = 5

TF_RAMP = 0
TF_KNOTS4 = 1

FOV_Y_DEG = 50.0
NEAR = 0.1
ORBIT_RADIUS = 1.5
GRID_K = 8
GRID_NZ = 20


# ----------------------------------------------------------------------------
# Cameras
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Camera:
    """Pinhole camera; values are float32 on purpose (both consumers widen the
    same float32 numbers)."""

    eye: Sequence[float]
    target: Sequence[float]
    up: Sequence[float]
    fov_y_deg: float = FOV_Y_DEG
    near: float = NEAR

    def as_array(self) -> np.ndarray:
        """eye[3], target[3], up[3], fov_y_deg, near as float32[11]."""
        return np.array(list(self.eye) + list(self.target) + list(self.up) + [self.fov_y_deg, self.near],
                        dtype=np.float32)


def orbit_camera(theta_deg: float, base_deg: float = 0.0, radius: float = ORBIT_RADIUS) -> Camera:
    """Camera on a circle about the volume centre (the y axis), facing the
    centre: eye = Rot_y(base + theta) (0, 0, radius).  V_N poses are rotations
    about the dataset centre, facing it (paper Section 5)."""
    a = math.radians(base_deg + theta_deg)
    eye = np.array([radius * math.sin(a), 0.0, radius * math.cos(a)], dtype=np.float32)
    return Camera(eye=tuple(float(x) for x in eye), target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0))


def aabb_for(dims) -> tuple:
    """AABB centred at the origin whose longest side is 1 (dims = nx, ny, nz)."""
    m = float(max(dims))
    half = [0.5 * d / m for d in dims]
    return tuple(-h for h in half), tuple(half)


def grid_z_for(cam: Camera, bmin, bmax, nz: int = GRID_NZ, pad: float = 1e-3) -> np.ndarray:
    """nz+1 float32 depth-slice boundaries, equal in view depth, spanning the
    V_O depths of the AABB corners padded by `pad` on each side."""
    eye = np.array(cam.eye, dtype=np.float64)
    F = np.array(cam.target, dtype=np.float64) - eye
    F /= np.linalg.norm(F)
    zs = []
    for cx in (bmin[0], bmax[0]):
        for cy in (bmin[1], bmax[1]):
            for cz in (bmin[2], bmax[2]):
                zs.append(float(F @ (np.array([cx, cy, cz]) - eye)))
    lo, hi = min(zs) - pad, max(zs) + pad
    return np.linspace(lo, hi, nz + 1).astype(np.float32)


# ----------------------------------------------------------------------------
# VDI container (plain data)
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class VDI:
    width: int
    height: int
    ns: int
    camera: Camera
    bmin: tuple
    bmax: tuple
    count: np.ndarray          # uint8 [H, W]
    depth: np.ndarray          # float32 [NS, H, W, 2]  (front, back) linear view depth
    rgba: np.ndarray           # float32 [NS, H, W, 4]  straight colour + opacity
    grid_k: int = GRID_K
    grid_nz: int = GRID_NZ
    grid_z: Optional[np.ndarray] = None   # float32 [grid_nz + 1]
    dvr: Optional[np.ndarray] = None      # float64 [H, W, 4] generator DVR composite (pins only)
    gamma: Optional[np.ndarray] = None    # float64 [H, W]
    nuncapped: Optional[np.ndarray] = None  # int32 [H, W]
    name: str = ""

    def __post_init__(self):
        # The bounds travel as float32 through the C ABI; keep exactly those values.
        self.bmin = tuple(float(np.float32(x)) for x in self.bmin)
        self.bmax = tuple(float(np.float32(x)) for x in self.bmax)
        if self.grid_z is None:
            self.grid_z = grid_z_for(self.camera, self.bmin, self.bmax, self.grid_nz)

    @property
    def nbytes_fp32(self) -> int:
        return self.width * self.height * self.ns * 24


# ----------------------------------------------------------------------------
# Native generator
# ----------------------------------------------------------------------------
_lib = None


def build(force: bool = False) -> str:
    """Compile the generator (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=gnu11", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.vg_volume_blobs.argtypes = [ctypes.c_int] * 4 + [P, P, P, P]
        lib.vg_volume_slab_u16.argtypes = [ctypes.c_int] * 3 + [ctypes.c_uint64, P]
        lib.vg_volume_shell_f32.argtypes = [ctypes.c_int] * 3 + [ctypes.c_uint64, P]
        lib.vg_generate.argtypes = ([ctypes.c_int] * 4 + [P, P, P, P] + [ctypes.c_int] * 4 +
                                    [ctypes.c_double] + [P] * 6)
        lib.vg_generate.restype = ctypes.c_int64
        lib.vg_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def volume_blobs(seed: int, n: int = 64, nblob: int = 8) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = np.ascontiguousarray(rng.uniform(8.0, n - 8.0, size=(nblob, 3)))
    sigmas = np.ascontiguousarray(rng.uniform(4.0, 12.0, size=nblob))
    amps = np.ascontiguousarray(rng.uniform(0.3, 1.0, size=nblob))
    out = np.empty((n, n, n), dtype=np.float32)
    _load().vg_volume_blobs(n, n, n, nblob, _ptr(centres), _ptr(sigmas), _ptr(amps), _ptr(out))
    return out


def volume_slab_u16(seed: int, dims=(512, 512, 512)) -> np.ndarray:
    nx, ny, nz = dims
    out = np.empty((nz, ny, nx), dtype=np.uint16)
    _load().vg_volume_slab_u16(nx, ny, nz, seed, _ptr(out))
    return out


def volume_shell_f32(seed: int, dims=(1024, 1024, 512)) -> np.ndarray:
    nx, ny, nz = dims
    out = np.empty((nz, ny, nx), dtype=np.float32)
    _load().vg_volume_shell_f32(nx, ny, nz, seed, _ptr(out))
    return out


def generate_vdi(volume: np.ndarray, camera: Camera, width: int, height: int, ns: int, tf: int,
                 gamma: float = 0.0, name: str = "") -> VDI:
    """Generate a VDI from a volume ([nz, ny, nx], float32 in [0,1] or uint16).
    gamma > 0: fixed sensitivity; gamma == 0: per-ray bisection (Alg. S1)."""
    if not (1 <= ns <= 255):
        raise ValueError("ns must be in [1, 255]")
    volume = np.ascontiguousarray(volume)
    nz, ny, nx = volume.shape
    is_u16 = 1 if volume.dtype == np.uint16 else 0
    if not is_u16 and volume.dtype != np.float32:
        raise TypeError("volume must be float32 or uint16")
    bmin, bmax = aabb_for((nx, ny, nz))
    bmin_a = np.array(bmin, dtype=np.float64)
    bmax_a = np.array(bmax, dtype=np.float64)
    cam = camera.as_array().astype(np.float64)
    count = np.empty((height, width), dtype=np.uint8)
    depth = np.empty((ns, height, width, 2), dtype=np.float32)
    rgba = np.empty((ns, height, width, 4), dtype=np.float32)
    dvr = np.empty((height, width, 4), dtype=np.float64)
    gam = np.empty((height, width), dtype=np.float64)
    nunc = np.empty((height, width), dtype=np.int32)
    _load().vg_generate(nx, ny, nz, is_u16, _ptr(volume), _ptr(bmin_a), _ptr(bmax_a), _ptr(cam),
                        width, height, ns, tf, float(gamma), _ptr(count), _ptr(depth), _ptr(rgba),
                        _ptr(dvr), _ptr(gam), _ptr(nunc))
    return VDI(width=width, height=height, ns=ns, camera=camera, bmin=bmin, bmax=bmax, count=count,
               depth=depth, rgba=rgba, dvr=dvr, gamma=gam, nuncapped=nunc, name=name)


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------
WORKLOADS = {
    "tiny": dict(volume="blobs", dims=(64, 64, 64), width=128, height=128, ns=16, tf=TF_RAMP, gamma=0.05,
                 seed=1001, angles=(0.0, 5.0)),
    "720p": dict(volume="slab_u16", dims=(512, 512, 512), width=1280, height=720, ns=20, tf=TF_KNOTS4,
                 gamma=0.0, seed=1002, angles=(0.0, 5.0, 10.0, 20.0, 30.0)),
    "1080p": dict(volume="shell_f32", dims=(1024, 1024, 512), width=1920, height=1080, ns=50, tf=TF_KNOTS4,
                  gamma=0.0, seed=1003, angles=tuple(5.0 * i for i in range(10))),
}


def cache_dir() -> str:
    d = os.environ.get("VDI_CACHE_DIR", os.path.join(_REPO, "_cache"))
    os.makedirs(d, exist_ok=True)
    return d


def make_volume(spec: dict) -> np.ndarray:
    kind = spec["volume"]
    if kind == "blobs":
        return volume_blobs(spec["seed"], spec["dims"][0])
    if kind == "slab_u16":
        return volume_slab_u16(spec["seed"], spec["dims"])
    if kind == "shell_f32":
        return volume_shell_f32(spec["seed"], spec["dims"])
    raise KeyError(kind)


def _key(spec: dict, base_deg: float) -> str:
    blob = json.dumps({"spec": {k: v for k, v in spec.items() if k != "angles"}, "base": base_deg,
                       "version": GENERATOR_VERSION}, sort_keys=True)
    return hashlib.sha1(blob.encode()).hexdigest()[:16]


def load_workload(name: str, base_deg: float = 0.0, verbose: bool = False, keep_dvr: bool = True) -> VDI:
    """VDI of a named workload with V_O at `base_deg` about y; generated once
    and cached on disk (VDI_CACHE_DIR, default <repo>/_cache)."""
    spec = WORKLOADS[name]
    key = _key(spec, base_deg)
    d = os.path.join(cache_dir(), f"{name}_{int(round(base_deg))}_{key}")
    cam = orbit_camera(0.0, base_deg)
    files = ["count", "depth", "rgba", "dvr", "gamma", "nuncapped"]
    if os.path.exists(os.path.join(d, "done")):
        arrs = {f: np.load(os.path.join(d, f + ".npy"), mmap_mode=None) for f in files
                if f in ("count", "depth", "rgba") or keep_dvr}
        bmin, bmax = aabb_for(spec["dims"])
        return VDI(width=spec["width"], height=spec["height"], ns=spec["ns"], camera=cam, bmin=bmin, bmax=bmax,
                   count=arrs["count"], depth=arrs["depth"], rgba=arrs["rgba"], dvr=arrs.get("dvr"),
                   gamma=arrs.get("gamma"), nuncapped=arrs.get("nuncapped"), name=name)
    t = time.time()
    vol = make_volume(spec)
    if verbose:
        print(f"[inputs] {name}: volume {vol.shape} {vol.dtype} in {time.time() - t:.1f}s", file=sys.stderr, flush=True)
    t = time.time()
    vdi = generate_vdi(vol, cam, spec["width"], spec["height"], spec["ns"], spec["tf"], spec["gamma"], name=name)
    del vol
    if verbose:
        print(f"[inputs] {name}: VDI {spec['width']}x{spec['height']}x{spec['ns']} in {time.time() - t:.1f}s, "
              f"{int(vdi.count.sum())} supersegments", file=sys.stderr, flush=True)
    tmp = d + ".tmp%d" % os.getpid()
    os.makedirs(tmp, exist_ok=True)
    for f in files:
        np.save(os.path.join(tmp, f + ".npy"), getattr(vdi, f))
    open(os.path.join(tmp, "done"), "w").close()
    try:
        os.replace(tmp, d)
    except OSError:
        pass
    return vdi


def generator_threads() -> int:
    return int(_load().vg_threads())
