"""GPU DVR (vdi_dvr) and image quality (vdi_image_quality), needs an MI355X.

- FP64 DVR against the CPU generator's FP64 DVR of the same view (same
  samples, same order): bit-identical after rounding to float32.
- FP32-shading DVR against the same reference: within 1e-4 (the render
  tolerance; accumulated FP32 rounding over up to 2 max(n) samples).
- SSIM / PSNR kernels against the FP64 numpy oracle (pinned in
  test_quality_pins.py) on random images and on VDI-vs-DVR images.
- A VDI rendered from its own generating view reproduces the DVR of that view
  (the supersegments hold the same samples, composited in the same order).
"""
import sys

import numpy as np
import pytest

import inputs
from oracle import quality as Q

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _V():
    from paper_2206_08660_amd import vdi as V
    return V


def to_device(vol):
    return torch.from_numpy(vol.view(np.int16) if vol.dtype == np.uint16 else vol).cuda()


TF_NAME = {inputs.TF_RAMP: "ramp", inputs.TF_KNOTS4: "knots4"}


def gpu_dvr(vol, dvol, cam, W, H, tf, precision):
    nz, ny, nx = vol.shape
    bmin, bmax = inputs.aabb_for((nx, ny, nz))
    img = _V().dvr(dvol, bmin, bmax, cam, W, H, tf=TF_NAME[tf], precision=precision)
    torch.cuda.synchronize()
    return img.cpu().numpy()


def ref_dvr(vol, cam, W, H, tf):
    # The generator's DVR does not depend on N_S or gamma; a large fixed gamma keeps the split cheap.
    return inputs.generate_vdi(vol, cam, W, H, 1, tf, gamma=10.0).dvr


@pytest.mark.parametrize("name,yaw,W,H", [("tiny", 17.0, 130, 97), ("720p", 20.0, 1280, 720), ("720p", 45.0, 64, 1)])
def test_dvr_matches_cpu_generator(name, yaw, W, H):
    spec = inputs.WORKLOADS[name]
    vol = inputs.make_volume(spec)
    dvol = to_device(vol)
    cam = inputs.orbit_camera(yaw)
    say(f"[gpu] DVR {name} yaw {yaw} {W}x{H}")
    ref = ref_dvr(vol, cam, W, H, spec["tf"])
    got = gpu_dvr(vol, dvol, cam, W, H, spec["tf"], "f64")
    bad = int((got.view(np.uint32) != ref.astype(np.float32).view(np.uint32)).any(axis=-1).sum())
    f32 = gpu_dvr(vol, dvol, cam, W, H, spec["tf"], "f32")
    err = float(np.abs(f32 - ref).max())
    say(f"[gpu]   FP64 pixels differing from the CPU generator: {bad}; FP32 shading max|d| {err:.2e}")
    assert bad == 0
    assert err <= 1e-4


def test_dvr_edge_cases():
    vol = inputs.make_volume(inputs.WORKLOADS["tiny"])
    dvol = to_device(vol)
    # Eye inside the volume (near-plane clipping) and a wide field of view (rays that miss).
    for cam in (inputs.orbit_camera(30.0, radius=0.2),
                inputs.Camera(eye=(0.0, 0.0, 1.5), target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), fov_y_deg=120.0)):
        ref = ref_dvr(vol, cam, 96, 64, inputs.TF_RAMP)
        got = gpu_dvr(vol, dvol, cam, 96, 64, inputs.TF_RAMP, "f64")
        assert np.array_equal(got, ref.astype(np.float32))
    empty = np.zeros((9, 10, 11), np.float32)
    assert not gpu_dvr(empty, to_device(empty), inputs.orbit_camera(5.0), 33, 17, inputs.TF_KNOTS4, "f32").any()


def test_quality_kernels_match_oracle():
    V = _V()
    rng = np.random.default_rng(4)
    for (H, W) in [(11, 11), (37, 70), (300, 257)]:
        a = rng.random((H, W, 4)).astype(np.float32)
        b = np.clip(a + 0.05 * rng.standard_normal(a.shape), 0, 1).astype(np.float32)
        s, p = V.image_quality(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda())
        say(f"[gpu] quality {W}x{H}: ssim {s:.6f} psnr {p:.3f}")
        assert s == pytest.approx(Q.ssim(a, b), abs=1e-10)
        assert p == pytest.approx(Q.psnr(a, b), abs=1e-9)
        s1, p1 = V.image_quality(torch.from_numpy(a).cuda(), torch.from_numpy(a).cuda())
        assert s1 == pytest.approx(1.0, abs=1e-12) and p1 == float("inf")


def test_vdi_at_its_own_view_reproduces_dvr_and_quality_falls_with_angle():
    V = _V()
    spec = inputs.WORKLOADS["720p"]
    src = inputs.load_workload("720p", keep_dvr=False)
    vol = inputs.make_volume(spec)
    dvol = to_device(vol)
    W, H = spec["width"], spec["height"]
    res = {}
    with V.Vdi(src) as h:
        for yaw in (0.0, 10.0, 30.0):
            cam = inputs.orbit_camera(yaw)
            img = h.render(cam, W, H)
            ref = V.dvr(dvol, src.bmin, src.bmax, cam, W, H, tf="knots4", precision="f64")
            s, p = V.image_quality(img, ref)
            torch.cuda.synchronize()
            a, b = img.cpu().numpy(), ref.cpu().numpy()
            so, po = Q.ssim(a, b), Q.psnr(a, b)
            say(f"[gpu] 720p VDI vs DVR at {yaw:g} deg: SSIM {s:.5f} (oracle {so:.5f}), PSNR {p:.2f} dB (oracle {po:.2f})")
            assert s == pytest.approx(so, abs=1e-9) and p == pytest.approx(po, abs=1e-7)
            res[yaw] = (s, p, float(np.abs(a - b).max()))
    assert res[0.0][2] <= 1e-4      # same samples in the same order at the generating view
    assert res[0.0][0] > 0.9999
    assert res[0.0][1] > res[10.0][1] > res[30.0][1]
