"""The GPU generator's per-ray code compiled for the host (hipcc, no GPU)
against the CPU FP64 generator: bit-identical counts, gammas, depths and
colours, with no sample cache, a cache shorter than the rays (the fallback
that samples the volume again), and a cache that holds every sample."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import inputs
from paper_2206_08660_amd import vdi as V

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2206_08660_amd", "csrc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("genhost") / "libgen_host.so")
    cmd = ["hipcc", "--offload-arch=gfx950", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, os.path.join(HERE, "host", "gen_host.hip"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    L = ctypes.CDLL(out)
    L.host_generate.argtypes = [ctypes.POINTER(V.Volume), ctypes.POINTER(V.GenParams)] + [ctypes.c_void_p] * 4 + \
        [ctypes.c_int]
    return L


def run_host(L, vol, cam, W, H, ns, tf, gamma, K):
    nz, ny, nx = vol.shape
    bmin, bmax = inputs.aabb_for((nx, ny, nz))
    v = V.Volume(nx, ny, nz, 1 if vol.dtype == np.uint16 else 0, ctypes.c_void_p(vol.ctypes.data))
    v.aabb_min[:] = bmin
    v.aabb_max[:] = bmax
    p = V.GenParams()
    p.camera_VO = V.camera(cam)
    p.width, p.height, p.max_supersegments, p.tf, p.gamma = W, H, ns, tf, gamma
    count = np.zeros((H, W), np.uint8)
    depth = np.zeros((ns, H, W, 2), np.float32)
    rgba = np.zeros((ns, H, W, 4), np.float32)
    gam = np.zeros((H, W))
    assert L.host_generate(ctypes.byref(v), ctypes.byref(p), count.ctypes.data, depth.ctypes.data,
                           rgba.ctypes.data, gam.ctypes.data, K) == 0
    return count, depth, rgba, gam


@pytest.mark.parametrize("K", [0, 37, 4096])
def test_host_build_matches_cpu_generator(harness, K):
    spec = inputs.WORKLOADS["720p"]
    vol = inputs.volume_slab_u16(spec["seed"], (96, 96, 96))
    for cam, W, H, ns, tf, gamma in [(inputs.orbit_camera(0.0), 80, 45, 20, inputs.TF_KNOTS4, 0.0),
                                     (inputs.orbit_camera(33.0), 57, 31, 6, inputs.TF_RAMP, 0.0),
                                     (inputs.orbit_camera(-20.0, radius=0.3), 40, 30, 9, inputs.TF_KNOTS4, 0.01)]:
        ref = inputs.generate_vdi(vol, cam, W, H, ns, tf, gamma)
        count, depth, rgba, gam = run_host(harness, vol, cam, W, H, ns, tf, gamma, K)
        assert ref.count.sum() > 0
        assert np.array_equal(count, ref.count) and np.array_equal(gam, ref.gamma)
        assert np.array_equal(depth.view(np.uint32), ref.depth.view(np.uint32))
        assert np.array_equal(rgba.view(np.uint32), ref.rgba.view(np.uint32))
