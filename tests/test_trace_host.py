"""The renderer's per-ray code compiled for the host (hipcc; nothing runs on
a GPU): exact rays with every first-supersegment search, with and without
empty-space skipping, and preview rays split into 1, 2, 4 or 8 blocks of grid
cells combined in the kernel's order, against the FP64 oracle (the count
grid comes from the oracle)."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import inputs
import oracle
from paper_2206_08660_amd import vdi as V
from tests import synth
from tests.gpu_util import TOL, tie_aware_errors

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def host(tmp_path_factory):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("renderhost") / "librender_host.so")
    cmd = ["hipcc", "--offload-arch=gfx950", "-O2", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_2206_08660_amd", "csrc"),
           os.path.join(HERE, "host", "render_host.hip"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    L = ctypes.CDLL(out)
    L.host_render.argtypes = [ctypes.POINTER(V.Desc), ctypes.c_void_p, ctypes.POINTER(V.Camera), ctypes.c_int,
                              ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_float, ctypes.c_int,
                              ctypes.c_void_p]
    return L


def render(L, src, cam, W, H, preview=False, search="window", ess=True, d_r=0.0, parts=0):
    d, keep = V._desc(src, "f32", False, None, "f32")
    grid = np.ascontiguousarray(oracle.count_grid(src), dtype=np.uint32)
    gz = np.ascontiguousarray(src.grid_z, dtype=np.float32)
    d.grid_z = gz.ctypes.data
    out = np.zeros((H, W, 4), np.float32)
    c = V.camera(cam)
    rc = L.host_render(ctypes.byref(d), grid.ctypes.data, ctypes.byref(c), W, H, int(preview), V.SEARCH[search],
                       int(ess), d_r, parts, out.ctypes.data)
    assert rc == 0
    return out.astype(np.float64)


@pytest.fixture(scope="module")
def tiny():
    return inputs.load_workload("tiny", keep_dvr=False)


@pytest.mark.parametrize("theta", [7.0, -33.0, 120.0])
def test_exact_every_search_and_skipping(host, tiny, theta):
    cam = inputs.orbit_camera(theta)
    ref = oracle.render_exact(tiny, cam, 64, 48)
    for ess in (True, False):
        for search in ("window", "seeded", "binary", "linear"):
            img = render(host, tiny, cam, 64, 48, search=search, ess=ess)
            assert np.abs(img - ref).max() <= TOL, (ess, search)


def test_exact_generating_view_with_skipping(host, tiny):
    """From V_O itself at V_O's resolution every ray stays in its own list:
    with skipping on, a ray in an empty grid cell takes the list step (one
    step to the list's exit) rather than one cell step per depth slice."""
    cam = tiny.camera
    ref = oracle.render_exact(tiny, cam, tiny.width, tiny.height)
    for ess in (True, False):
        img = render(host, tiny, cam, tiny.width, tiny.height, ess=ess)
        assert np.abs(img - ref).max() <= TOL, ess


def test_exact_random_vdi(host):
    v = synth.random_vdi(30, 20, 9, seed=12)
    for theta in (25.0, 135.0):
        cam = inputs.orbit_camera(theta)
        ref = oracle.render_exact(v, cam, 40, 26)
        assert np.abs(render(host, v, cam, 40, 26) - ref).max() <= TOL


@pytest.mark.parametrize("ns,seed", [(70, 3), (255, 4)])
def test_exact_long_lists(host, ns, seed):
    """Lists of every length from 0 to N_S, up to 255, thin supersegments
    (alpha <= 0.12, so rays pass many of them): the directory bracket, the
    bisection that narrows it for lists over about 60 slots, windows that
    continue past their end, forwards (3 and 25 deg) and backwards (135 deg),
    every search against the oracle."""
    v = synth.random_vdi(24, 16, ns, seed=seed, alpha_max=0.12, empty_frac=0.1)
    assert v.count.max() > 60 and (v.count <= 8).any()
    for theta in (3.0, 25.0, 135.0):
        cam = inputs.orbit_camera(theta)
        ref = oracle.render_exact(v, cam, 40, 26)
        assert (ref[..., 3] > 0).mean() > 0.5
        for search in ("window", "binary"):
            for ess in (True, False):
                img = render(host, v, cam, 40, 26, search=search, ess=ess)
                assert np.abs(img - ref).max() <= TOL, (theta, search, ess)


@pytest.mark.parametrize("theta", [9.0, 150.0])
@pytest.mark.parametrize("parts", [1, 2, 4, 8])
def test_preview_split_rays(host, tiny, parts, theta):
    """Rays moving away from V_O (9 deg) and towards it (150 deg)."""
    cam = inputs.orbit_camera(theta)
    ref, flags = oracle.render_preview(tiny, cam, 64, 48, 2.0)
    ok = flags == 0
    img = render(host, tiny, cam, 64, 48, preview=True, d_r=2.0, parts=parts)
    whole = render(host, tiny, cam, 64, 48, preview=True, d_r=2.0, parts=1)
    assert ok.mean() > 0.9
    assert np.abs(img - ref)[ok].max() <= TOL
    # The blocks take the whole ray's samples; only rounding and early termination differ.
    assert np.abs(img - whole).max() <= 1e-5


@pytest.mark.parametrize("d_i", [2, 4])
def test_preview_ties_resolved_one_way(host, tiny, d_i):
    """The downsampled preview from the generating viewpoint puts every
    low-res pixel centre on a V_O list edge (128 / 64 = 2, 128 / 32 = 4), so
    every sample of a ray is a tie.  The per-ray code must resolve them one
    way along the ray: every pixel, flagged or not, equals the oracle's
    unique result or one of its consistent tie resolutions."""
    cam = inputs.orbit_camera(0.0)
    w = h = 128 // d_i
    pix = np.arange(w * h)
    ref, flags = oracle.render_preview(tiny, cam, w, h, 2.0, pixels=pix)
    var = oracle.preview_tie_variants(tiny, cam, w, h, 2.0, pix[flags != 0])
    nonempty = ref[:, 3] > 0
    assert (nonempty & (flags != 0)).sum() >= 100
    for parts in (1, 2, 8):
        img = render(host, tiny, cam, w, h, preview=True, d_r=2.0, parts=parts).reshape(-1, 4)
        err, _ = tie_aware_errors(img, ref, flags, var)
        assert err.max() <= TOL, (parts, err.max())
        # The x and y list edges are resolved towards +x and +y.
        pos = [k for k, b in enumerate(oracle.TIE_BIASES) if b[0] == 1 and b[1] == 1]
        err_pos, _ = tie_aware_errors(img, ref, flags, var[pos])
        assert err_pos.max() <= TOL, (parts, err_pos.max())


# Rays whose equal-parameter cut lands on a corner of the count grid, where a
# list-grid line and a depth-slice face are crossed at the same parameter up
# to rounding: the lanes must take up the walk exactly where the previous one
# leaves it.  (yaw, width, height, D_R) of frames where cells were lost between
# two lanes when a lane's start came from point location alone.
CORNER_CASES = [(-36.37798448780438, 97, 61, 0.5), (161.61972297759553, 109, 16, 1.0),
                (-125.89939191785794, 97, 44, 0.25), (122.87422066045798, 25, 55, 0.5),
                (31.004303332583817, 97, 51, 0.25)]


@pytest.mark.parametrize("yaw,w,h,d_r", CORNER_CASES)
def test_preview_split_rays_at_grid_corners(host, tiny, yaw, w, h, d_r):
    cam = inputs.orbit_camera(yaw)
    whole = render(host, tiny, cam, w, h, preview=True, d_r=d_r, parts=1)
    ref, flags = oracle.render_preview(tiny, cam, w, h, d_r)
    assert np.abs(whole - ref)[flags == 0].max() <= TOL
    for parts in (2, 4, 8):
        img = render(host, tiny, cam, w, h, preview=True, d_r=d_r, parts=parts)
        # only early termination differs between the blocks and the whole ray
        assert np.abs(img - whole).max() <= 1.1e-5, parts


def test_preview_split_rays_random_views(host, tiny):
    """Seeded views in all directions, sizes and D_R: every split of every
    ray takes exactly the whole ray's samples."""
    rng = np.random.default_rng(20)
    rv = synth.random_vdi(30, 20, 9, seed=12)
    for case in range(16):
        src = tiny if case % 2 else rv
        yaw = float(rng.uniform(-180.0, 180.0))
        w, h = int(rng.integers(20, 90)), int(rng.integers(15, 60))
        d_r = float((0.25, 0.5, 1.0, 2.0)[case % 4])
        cam = inputs.orbit_camera(yaw)
        whole = render(host, src, cam, w, h, preview=True, d_r=d_r, parts=1)
        for parts in (2, 8):
            img = render(host, src, cam, w, h, preview=True, d_r=d_r, parts=parts)
            assert np.abs(img - whole).max() <= 1.1e-5, (case, yaw, w, h, d_r, parts)
