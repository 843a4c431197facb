"""GPU VDI generation (vdi_generate, needs an MI355X) against the CPU FP64
generator of `inputs` (Section 3, Eq. 1; supplement Alg. S1).

Both sides run the same FP64 steps in the same order without fused
multiply-adds, so supersegment counts, gammas, depths and colours are
compared bit for bit, on the full-size workloads and on edge cases: ragged
sizes, N_S = 1 (everything in one smeared supersegment), an eye inside the
volume (near-plane clipping), an empty volume and rays that miss it.
"""
import sys

import numpy as np
import pytest

import inputs

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


def to_device(vol):
    if vol.dtype == np.uint16:
        return torch.from_numpy(vol.view(np.int16)).cuda()
    return torch.from_numpy(vol).cuda()


def gpu_generate(dvol, cam, W, H, ns, tf, gamma, bmin=None, bmax=None):
    from paper_2206_08660_amd import vdi as V
    nz, ny, nx = dvol.shape
    if bmin is None:
        bmin, bmax = inputs.aabb_for((nx, ny, nz))
    count, depth, rgba, gam = V.generate(dvol, bmin, bmax, cam, W, H, ns, tf={0: "ramp", 1: "knots4"}[tf],
                                         gamma=gamma)
    torch.cuda.synchronize()
    return count.cpu().numpy(), depth.cpu().numpy(), rgba.cpu().numpy(), gam.cpu().numpy()


def check_same(tag, ref, got):
    count, depth, rgba, gam = got
    bad = {
        "count": int((count != ref.count).sum()),
        "gamma": int((gam != ref.gamma).sum()),
        "depth": int((depth.view(np.uint32) != ref.depth.view(np.uint32)).any(axis=-1).sum()),
        "rgba": int((rgba.view(np.uint32) != ref.rgba.view(np.uint32)).any(axis=-1).sum()),
    }
    say(f"[gpu] {tag}: {int(ref.count.sum())} supersegments in {ref.count.size} lists, mismatches {bad}")
    assert all(v == 0 for v in bad.values()), (tag, bad)


@pytest.fixture(scope="module")
def tiny_vol():
    return inputs.make_volume(inputs.WORKLOADS["tiny"])


@pytest.mark.parametrize("yaw", [0.0, 37.0])
def test_tiny_fixed_gamma(tiny_vol, yaw):
    spec = inputs.WORKLOADS["tiny"]
    cam = inputs.orbit_camera(yaw)
    say(f"[gpu] generate tiny yaw {yaw}")
    ref = inputs.generate_vdi(tiny_vol, cam, spec["width"], spec["height"], spec["ns"], spec["tf"], spec["gamma"])
    check_same(f"tiny yaw {yaw}", ref, gpu_generate(to_device(tiny_vol), cam, spec["width"], spec["height"],
                                                       spec["ns"], spec["tf"], spec["gamma"]))


@pytest.mark.parametrize("W,H,ns,tf,gamma", [(100, 70, 3, inputs.TF_RAMP, 0.0), (65, 1, 1, inputs.TF_KNOTS4, 0.0),
                                             (1, 33, 7, inputs.TF_RAMP, 0.02), (130, 96, 255, inputs.TF_RAMP, 0.0)])
def test_ragged_and_extreme_ns(tiny_vol, W, H, ns, tf, gamma):
    cam = inputs.orbit_camera(12.0)
    say(f"[gpu] generate tiny {W}x{H} ns {ns} tf {tf} gamma {gamma}")
    ref = inputs.generate_vdi(tiny_vol, cam, W, H, ns, tf, gamma)
    check_same(f"{W}x{H} ns {ns}", ref, gpu_generate(to_device(tiny_vol), cam, W, H, ns, tf, gamma))


def test_eye_inside_volume_and_empty_volume(tiny_vol):
    cam = inputs.orbit_camera(20.0, radius=0.2)  # inside the AABB: the near plane clips
    say("[gpu] generate with the eye inside the volume")
    ref = inputs.generate_vdi(tiny_vol, cam, 96, 64, 12, inputs.TF_RAMP, 0.0)
    check_same("eye inside", ref, gpu_generate(to_device(tiny_vol), cam, 96, 64, 12, inputs.TF_RAMP, 0.0))
    empty = np.zeros((20, 24, 16), dtype=np.float32)
    cam = inputs.orbit_camera(45.0)
    say("[gpu] generate from an empty volume")
    ref = inputs.generate_vdi(empty, cam, 80, 40, 5, inputs.TF_KNOTS4, 0.0)
    got = gpu_generate(to_device(empty), cam, 80, 40, 5, inputs.TF_KNOTS4, 0.0)
    check_same("empty", ref, got)
    assert got[0].sum() == 0 and not got[1].any() and not got[2].any()
    # Wide field of view: the outer rays miss the volume (count 0, gamma 0).
    cam = inputs.Camera(eye=(0.0, 0.0, 1.5), target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), fov_y_deg=120.0)
    ref = inputs.generate_vdi(tiny_vol, cam, 64, 64, 8, inputs.TF_RAMP, 0.0)
    got = gpu_generate(to_device(tiny_vol), cam, 64, 64, 8, inputs.TF_RAMP, 0.0)
    check_same("wide fov", ref, got)
    assert (got[3] == 0.0).any() and (got[0] == 0).any()


def test_720p_workload_full_size():
    spec = inputs.WORKLOADS["720p"]
    vol = inputs.make_volume(spec)
    dvol = to_device(vol)
    for yaw in (0.0, 30.0):
        cam = inputs.orbit_camera(yaw)
        say(f"[gpu] generate 720p yaw {yaw}")
        ref = inputs.generate_vdi(vol, cam, spec["width"], spec["height"], spec["ns"], spec["tf"], spec["gamma"])
        check_same(f"720p yaw {yaw}", ref, gpu_generate(dvol, cam, spec["width"], spec["height"], spec["ns"],
                                                           spec["tf"], spec["gamma"]))


def test_1080p_workload_full_size():
    """The 1080p workload's VDI (the renderer's benchmark input) regenerated on the GPU."""
    spec = inputs.WORKLOADS["1080p"]
    say("[gpu] loading the 1080p workload")
    ref = inputs.load_workload("1080p", verbose=True)
    vol = inputs.make_volume(spec)
    dvol = to_device(vol)
    del vol
    say("[gpu] generate 1080p")
    got = gpu_generate(dvol, ref.camera, spec["width"], spec["height"], spec["ns"], spec["tf"], spec["gamma"])
    check_same("1080p", ref, got)


def test_generated_vdi_is_rendered_without_a_host_copy(tiny_vol):
    """vdi_generate's device planes go straight into vdi_create and
    vdi_replace_begin (planes_on_device): renders are bit-identical to those
    of the same VDI generated on the CPU and uploaded from host memory."""
    from paper_2206_08660_amd import vdi as V
    spec = inputs.WORKLOADS["tiny"]
    W0, H0, ns = spec["width"], spec["height"], spec["ns"]
    dvol = to_device(tiny_vol)
    bmin, bmax = inputs.aabb_for(tiny_vol.shape[::-1])

    def both(base):
        cam_o = inputs.orbit_camera(0.0, base)
        host = inputs.generate_vdi(tiny_vol, cam_o, W0, H0, ns, spec["tf"], 0.0)
        c, d, r, _ = V.generate(dvol, bmin, bmax, cam_o, W0, H0, ns, tf="ramp", gamma=0.0, gamma_out=False)
        return host, V.DeviceVDI(c, d, r, cam_o, host.bmin, host.bmax, grid_z=host.grid_z)

    host0, dev0 = both(0.0)
    host1, dev1 = both(25.0)
    views = [(inputs.orbit_camera(12.0), 1.0, 0.0), (inputs.orbit_camera(-20.0), 2.0, 1.5)]
    with V.Vdi(host0) as hh, V.Vdi(dev0) as hd:
        for cam, di, dr in views:
            a, b = hh.render(cam, 96, 80, di, dr), hd.render(cam, 96, 80, di, dr)
            torch.cuda.synchronize()
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
        assert hd.info().supersegments == int(host0.count.sum())
        # Replacement from device planes written on the caller's stream.
        hd.replace_begin(dev1)
        while not hd.replace_poll():
            pass
        with V.Vdi(host1) as h1:
            for cam, di, dr in views:
                a, b = h1.render(cam, 96, 80, di, dr), hd.render(cam, 96, 80, di, dr)
                torch.cuda.synchronize()
                assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    with pytest.raises(V.VdiError):
        V.Vdi(dev0, validate=True)   # list validation needs host planes


# ------------------------------------------------------- pins not through the CPU generator
from tests import slabs  # noqa: E402
from tests.synth import composite_at_vo  # noqa: E402


@pytest.mark.parametrize("side", [-1, 1])
def test_eq1_two_layers_closed_form_on_gpu(side):
    """Eq. 1 at an intermediate gamma on the GPU: the centre ray of a
    two-layer volume splits just below d = |c1 a1 - c2 a2| and merges just
    above it, with closed-form faces, colours and opacities."""
    runs = slabs.run(slabs.TWO)
    g = slabs.eq1_distance(runs[:1], slabs.TWO[1][0]) * (1.0 + side * 1e-6)
    count, depth, rgba, _ = gpu_generate(to_device(slabs.volume(slabs.TWO)), slabs.camera(), slabs.W, slabs.H, 4,
                                         inputs.TF_RAMP, g)
    slabs.check(count, depth, rgba, slabs.expected(slabs.TWO, g, 4))


@pytest.mark.parametrize("gamma,n", slabs.THREE_CASES)
def test_eq1_three_layers_on_gpu(gamma, n):
    count, depth, rgba, _ = gpu_generate(to_device(slabs.volume(slabs.THREE)), slabs.camera(), slabs.W, slabs.H, 8,
                                         inputs.TF_RAMP, gamma)
    want = slabs.expected(slabs.THREE, gamma, 8)
    assert len(want) == n
    slabs.check(count, depth, rgba, want)


def test_gamma_search_end_states_on_gpu():
    """The bracket search on layered rays (closed forms as in the CPU
    suite): the first trial stands at N_S = 2, the first midpoint at N_S = 1,
    the fourth midpoint for three layers at N_S = 2."""
    cam = slabs.camera()
    c, d, r, g = gpu_generate(to_device(slabs.volume(slabs.TWO)), cam, slabs.W, slabs.H, 2, inputs.TF_RAMP, 0.0)
    assert g[slabs.CY, slabs.CX] == 1e-5 and c[slabs.CY, slabs.CX] == 2
    c, d, r, g = gpu_generate(to_device(slabs.volume(slabs.TWO)), cam, slabs.W, slabs.H, 1, inputs.TF_RAMP, 0.0)
    assert abs(g[slabs.CY, slabs.CX] - 0.5 * (1e-5 + 3.0 ** 0.5)) < 1e-12
    slabs.check(c, d, r, slabs.expected(slabs.TWO, 1.0, 1))
    c, d, r, g = gpu_generate(to_device(slabs.volume(slabs.THREE)), cam, slabs.W, slabs.H, 2, inputs.TF_RAMP, 0.0)
    assert abs(g[slabs.CY, slabs.CX] - slabs.searched_gamma_three()) < 1e-12
    slabs.check(c, d, r, slabs.expected(slabs.THREE, float(g[slabs.CY, slabs.CX]), 2))


def test_720p_generated_vdi_invariants_on_gpu():
    """On the GPU's own 720p VDI (N_S = 20): its composite from V_O equals
    the GPU's FP64 DVR of the volume within 2e-6 (compositing inside a
    supersegment is exact, smearing included); every count is at most N_S;
    every searched ray ends with its first trial (gamma = 1e-5) or with a
    count in [N_S - delta, N_S], but for the rare rays whose bracket closed
    between two counts (at most 0.1% of the rays that hit)."""
    from paper_2206_08660_amd import vdi as V
    spec = inputs.WORKLOADS["720p"]
    vol = inputs.make_volume(spec)
    dvol = to_device(vol)
    del vol
    nz, ny, nx = dvol.shape
    bmin, bmax = inputs.aabb_for((nx, ny, nz))
    W, H, ns = spec["width"], spec["height"], spec["ns"]
    cam = inputs.orbit_camera(0.0)
    count, depth, rgba, gam = gpu_generate(dvol, cam, W, H, ns, spec["tf"], 0.0)
    dvr = V.dvr(dvol, bmin, bmax, cam, W, H, tf="knots4", precision="f64")
    torch.cuda.synchronize()
    dvr = dvr.cpu().numpy().astype(np.float64)
    v = inputs.VDI(width=W, height=H, ns=ns, camera=cam, bmin=bmin, bmax=bmax, count=count, depth=depth, rgba=rgba)
    comp = composite_at_vo(v)
    err = float(np.abs(comp - dvr).max())
    say(f"[gpu] 720p generated VDI: composite vs FP64 DVR max |d| = {err:.2e}")
    assert err <= 2e-6
    assert (count <= ns).all()
    delta = int(0.15 * ns)
    hit = count > 0
    first = gam == 1e-5
    ok = first | ((count >= ns - delta) & (count <= ns))
    assert (hit & ~ok).sum() <= 1e-3 * hit.sum()
    assert hit.sum() > 100000
