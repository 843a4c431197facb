"""vdi_render_noalloc (the allocation-free form of vdi_render) against
vdi_render, through the C ABI (needs an MI355X).

Both entry points run the same kernels; the allocation-free one keeps the
low-res image of a downsampled render in the library's static device array
instead of pool scratch.  Two calls in a row, the second smaller, must each
give vdi_render's image bit for bit (the array keeps the first call's texels
beyond the second's), and images within 1e-4 of the FP64 oracle."""
import sys

import numpy as np
import pytest

import inputs
import oracle
from tests.gpu_util import TOL, exact_errors, preview_errors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tiny_vdi():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    from paper_2206_08660_amd import vdi as V
    src = inputs.load_workload("tiny")
    h = V.Vdi(src)
    yield src, h
    torch.cuda.synchronize()
    h.close()


def _both(h, cam, W, H, d_i, d_r):
    a = h.render_noalloc(cam, W, H, d_i=d_i, d_r=d_r)
    b = h.render(cam, W, H, d_i=d_i, d_r=d_r)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


def test_noalloc_matches_render_two_calls_second_smaller(tiny_vdi):
    src, h = tiny_vdi
    cam = inputs.orbit_camera(12.0)
    # First call: 1000 x 800 at D_I = 2 (a 500 x 400 low-res preview image);
    # second: 300 x 210 at D_I = 3 (exact mode on a 100 x 70 grid).  Both
    # low-res grids keep the display's aspect, so rendering them directly
    # casts the rays of the D_I frame.
    for (W, H, d_i, d_r) in [(1000, 800, 2.0, 2.0), (300, 210, 3.0, 0.0)]:
        say(f"[gpu] noalloc {W}x{H} D_I={d_i} D_R={d_r}")
        a, b = _both(h, cam, W, H, d_i, d_r)
        assert np.array_equal(a, b), float(np.abs(a - b).max())
        # The low-res image itself against the oracle, ties included.
        w, hh = oracle.lowres_size(W, H, d_i)
        assert w * H == hh * W
        lo = h.render_noalloc(cam, w, hh, d_r=d_r).cpu().numpy().astype(np.float64).reshape(-1, 4)
        pix = np.random.default_rng(W).choice(w * hh, min(w * hh, 3000), replace=False)
        if d_r > 0:
            err, _, ref = preview_errors(lo[pix], src, cam, w, hh, d_r, pix, aspect=W / H)
        else:
            err, _, ref = exact_errors(lo[pix], src, cam, w, hh, pix, aspect=W / H)
        assert err.max() <= TOL and (ref[:, 3] > 0).sum() >= 300
        up = oracle.upsample(lo.reshape(hh, w, 4), W, H)[0]
        assert np.abs(a - up).max() <= 1e-6


def test_noalloc_exact_full_resolution(tiny_vdi):
    src, h = tiny_vdi
    cam = inputs.orbit_camera(-20.0)
    a, b = _both(h, cam, 128, 128, 1.0, 0.0)
    assert np.array_equal(a, b)
    assert np.abs(a - oracle.render_exact(src, cam, 128, 128)).max() <= TOL


def test_noalloc_allocates_no_device_memory(tiny_vdi):
    """After the first call on the device, further calls at new low-res
    sizes leave the device's free memory unchanged (vdi_render's pool would
    map new blocks for them)."""
    src, h = tiny_vdi
    cam = inputs.orbit_camera(7.0)
    sizes = [(640, 480, 1.5, 1.0), (1600, 1200, 1.1, 2.0), (64, 48, 2.0, 0.0)]
    outs = [torch.empty((H, W, 4), dtype=torch.float32, device="cuda") for (W, H, _, _) in sizes]
    h.render_noalloc(cam, 32, 32, d_i=2.0, d_r=1.0)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for (W, H, d_i, d_r), o in zip(sizes, outs):
        h.render_noalloc(cam, W, H, d_i=d_i, d_r=d_r, out=o)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)


def test_noalloc_rejects_low_res_beyond_scratch(tiny_vdi):
    from paper_2206_08660_amd import vdi as V
    src, h = tiny_vdi
    cam = inputs.orbit_camera(0.0)
    out = torch.empty((3000, 4000, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(V.VdiError) as e:
        h.render_noalloc(cam, 4000, 3000, d_i=1.5, d_r=1.0, out=out)   # 2667 x 2000 low-res texels
    assert e.value.code == V.VDI_ERR_ARG and "scratch" in str(e.value)
    # 2048 x 1024 = the maximum, accepted.
    out = torch.empty((2048, 4096, 4), dtype=torch.float32, device="cuda")
    h.render_noalloc(cam, 4096, 2048, d_i=2.0, d_r=4.0, out=out)
    torch.cuda.synchronize()
