"""Per-wavefront reuse of the exact walker's global loads (host replay,
tests/host/reuse_host.hip): the fraction of a wavefront's line requests that
an LRU cache of its own, of a given size, would serve.

    python -m tests.reuse_replay [row_step] [angles]

prints the table for the 1920x1080 frames of the 1080p VDI (N_S = 50) at the
given viewpoints, on every row_step-th row of 8x8 tiles (default 8; 5, 20, 45
degrees).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

from paper_2206_08660_amd import vdi as V  # noqa: E402

STREAMS = ("counts", "occupancy bits", "depth pairs", "colours")
# Capacities in 128-byte lines: about 1.3, 3.3, 6.5, 13, 26 and 52 KB, and unbounded.
CAPS = (10, 26, 52, 104, 208, 416, 1 << 30)


def build(out_dir: str | None = None) -> ctypes.CDLL:
    out_dir = out_dir or tempfile.mkdtemp(prefix="reuse_host_")
    out = os.path.join(out_dir, "libreuse_host.so")
    cmd = ["hipcc", "--offload-arch=gfx950", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_2206_08660_amd", "csrc"),
           os.path.join(HERE, "host", "reuse_host.hip"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    L = ctypes.CDLL(out)
    L.reuse_tile_trace.restype = ctypes.c_longlong
    L.reuse_tile_trace.argtypes = [ctypes.POINTER(V.Desc), ctypes.c_void_p, ctypes.POINTER(V.Camera), ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_longlong]
    L.reuse_exact.argtypes = [ctypes.POINTER(V.Desc), ctypes.c_void_p, ctypes.POINTER(V.Camera), ctypes.c_int,
                              ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    return L


def _desc(src):
    import oracle
    d, keep = V._desc(src, "f32", False, None, "f32")
    grid = np.ascontiguousarray(oracle.count_grid(src), dtype=np.uint32)
    gz = np.ascontiguousarray(src.grid_z, dtype=np.float32)
    d.grid_z = gz.ctypes.data
    return d, (keep, grid, gz)


def tile_trace(L, src, cam, W: int, H: int, tx: int, ty: int):
    """(lines, streams) of the requests of one exact tile, in issue order."""
    d, keep = _desc(src)
    c = V.camera(cam)
    n = L.reuse_tile_trace(ctypes.byref(d), keep[1].ctypes.data, ctypes.byref(c), W, H, tx, ty, None, None, 0)
    assert n >= 0
    lines = np.zeros(max(1, n), np.uint64)
    streams = np.zeros(max(1, n), np.int32)
    m = L.reuse_tile_trace(ctypes.byref(d), keep[1].ctypes.data, ctypes.byref(c), W, H, tx, ty, lines.ctypes.data,
                           streams.ctypes.data, n)
    assert m == n
    return lines[:n], streams[:n]


def replay(L, src, cam, W: int, H: int, row_step: int = 1, caps=CAPS):
    """stats[stream] = (requests, cold, hits at each capacity)."""
    d, keep = _desc(src)
    c = V.camera(cam)
    caps_a = np.asarray(caps, np.int32)
    st = np.zeros(4 * (2 + len(caps)))
    rc = L.reuse_exact(ctypes.byref(d), keep[1].ctypes.data, ctypes.byref(c), W, H, row_step, caps_a.ctypes.data,
                       len(caps), st.ctypes.data)
    assert rc == 0
    return st.reshape(4, 2 + len(caps))


def main():
    import inputs
    row_step = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    angles = [float(a) for a in sys.argv[2].split(",")] if len(sys.argv) > 2 else [5.0, 20.0, 45.0]
    L = build()
    src = inputs.load_workload("1080p", keep_dvr=False)
    print("hit fraction of a wavefront's line requests, LRU of its own of "
          + " / ".join(f"{c * 128 / 1024:.1f} KB" if c < 1 << 20 else "unbounded" for c in CAPS))
    for a in angles:
        st = replay(L, src, inputs.orbit_camera(a), src.width, src.height, row_step)
        print(f"{a:g} deg")
        for name, row in list(zip(STREAMS, st)) + [("all", st.sum(0))]:
            print(f"  {name:15s} requests {row[0]:11.0f}  cold {row[1] / row[0]:.3f}  hits "
                  + " ".join(f"{h / row[0]:.3f}" for h in row[2:]))


if __name__ == "__main__":
    main()
