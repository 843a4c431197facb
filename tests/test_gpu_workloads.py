"""HIP path vs the FP64 oracle on the full-size workloads (needs an MI355X).

Frames are rendered whole on the GPU in the configuration the benchmark
times (ESS on, window search); the oracle computes a stratified sample of
their pixels one by one.  Precision forms: FP16/BF16 colour storage against
the oracle fed the same rounded colours (<= 1e-4), and PSNR against the
oracle on the FP32 colours (>= 50 dB).
"""
import sys

import numpy as np
import pytest

import inputs
import oracle
from tests.gpu_util import TOL, nonempty_stratum, preview_errors, psnr, sample_pixels

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


def frame(h, cam, W, H, **kw):
    out = h.render(cam, W, H, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64).reshape(-1, 4)


@pytest.fixture(scope="module")
def w720():
    say("[gpu] loading 720p workload")
    return inputs.load_workload("720p", verbose=True)


@pytest.fixture(scope="module")
def w1080():
    say("[gpu] loading 1080p workload")
    return inputs.load_workload("1080p", verbose=True)


@pytest.fixture(scope="module")
def h720(w720):
    h = _V().Vdi(w720)
    yield h
    h.close()


@pytest.fixture(scope="module")
def h1080(w1080):
    h = _V().Vdi(w1080)
    yield h
    h.close()


def test_720p_grid_bit_exact(w720, h720):
    assert np.array_equal(h720.grid(), oracle.count_grid(w720))


@pytest.mark.parametrize("theta", [0.0, 5.0, 10.0, 20.0, 30.0])
def test_720p_exact_sampled(w720, h720, theta):
    say(f"[gpu] 720p exact theta={theta}")
    cam = inputs.orbit_camera(theta)
    pix = sample_pixels(1280, 720, 4000, seed=int(theta))
    ref = oracle.render_exact(w720, cam, 1280, 720, pixels=pix)
    img = frame(h720, cam, 1280, 720)
    assert np.abs(img[pix] - ref).max() <= TOL
    if theta == 20.0:
        for ess, search in [(True, "seeded"), (False, "window"), (True, "binary"), (True, "linear"), (False, "linear")]:
            other = frame(h720, cam, 1280, 720, ess=ess, search=search)
            assert np.abs(other - img).max() <= 1e-6, (ess, search)


def check_preview_workload(h, src, cam, W, H, d_i, d_r, n_texels, seed, min_nonempty):
    """A preview frame of the benchmark's kind, checked in two parts.
    Low-res image: the GPU renders the round(W/D_I) x round(H/D_I) ray grid
    directly (same rays, lane split and tile order as inside the D_I frame);
    sampled texels, a stratum of them non-empty, are compared with the
    oracle, texels that rest on ties with every consistent tie resolution.
    Upsampling: the GPU's W x H frame equals the oracle's bilinear upsampling
    of that GPU low-res image.  Returns the number of non-empty texels checked."""
    w, h_ = oracle.lowres_size(W, H, d_i)
    assert w * H == h_ * W, "the direct low-res render uses its own aspect, which must be the display's"
    lo = frame(h, cam, w, h_, d_r=d_r).reshape(h_, w, 4)
    full = frame(h, cam, W, H, d_i=d_i, d_r=d_r).reshape(H, W, 4)
    pix = np.unique(np.concatenate([sample_pixels(w, h_, n_texels, seed=seed),
                                    nonempty_stratum(lo, n_texels // 2, seed=seed)]))
    if d_r > 0:
        err, flags, ref = preview_errors(lo.reshape(-1, 4)[pix], src, cam, w, h_, d_r, pix, aspect=W / H)
    else:
        ref = oracle.render_exact(src, cam, w, h_, pixels=pix, aspect=W / H)
        err, flags = np.abs(lo.reshape(-1, 4)[pix] - ref).max(axis=1), np.zeros(len(pix), np.uint8)
    nonempty = int(((ref[:, 3] > 0) | (lo.reshape(-1, 4)[pix, 3] > 0)).sum())
    say(f"[gpu]   {len(pix)} texels of {w}x{h_}: {nonempty} non-empty, {int(flags.sum())} on ties; "
        f"max err {err.max():.2e}")
    assert err.max() <= TOL
    assert nonempty >= min_nonempty
    if (w, h_) != (W, H):
        up, _ = oracle.upsample(lo, W, H)
        assert np.abs(full - up).max() <= 1e-6
    else:
        assert np.array_equal(full, lo)
    assert np.isfinite(full).all() and full.min() >= 0.0 and full[..., 3].max() <= 1.0
    return nonempty


@pytest.mark.parametrize("theta,d_i,d_r", [(12.0, 2.0, 2.0), (35.0, 4.0, 1.0), (20.0, 1.0, 3.0), (0.0, 2.0, 2.0)])
def test_720p_preview_sampled(w720, h720, theta, d_i, d_r):
    """The dense slab, where rays terminate early: preview rays split over 2
    and 8 lanes (D_I = 2 and 4) composite each block from full transmittance,
    so a block behind the serial stop adds at most 1e-5."""
    say(f"[gpu] 720p preview theta={theta} D_I={d_i} D_R={d_r}")
    check_preview_workload(h720, w720, inputs.orbit_camera(theta), 1280, 720, d_i, d_r, 4000,
                           300 + int(theta), 1000)


def test_1080p_grid_bit_exact(w1080, h1080):
    assert np.array_equal(h1080.grid(), oracle.count_grid(w1080))


@pytest.mark.parametrize("theta", [5.0 * i for i in range(10)])
def test_1080p_exact_sampled(w1080, h1080, theta):
    say(f"[gpu] 1080p exact theta={theta}")
    cam = inputs.orbit_camera(theta)
    pix = sample_pixels(1920, 1080, 3000, seed=100 + int(theta))
    ref = oracle.render_exact(w1080, cam, 1920, 1080, pixels=pix)
    img = frame(h1080, cam, 1920, 1080)
    assert np.abs(img[pix] - ref).max() <= TOL


@pytest.mark.parametrize("theta,d_i,d_r", [(0.0, 2.0, 2.0), (0.0, 4.0, 2.0), (20.0, 2.0, 2.0), (45.0, 2.0, 2.0),
                                           (10.0, 4.0, 2.0), (30.0, 4.0, 2.0), (45.0, 4.0, 2.0), (25.0, 2.0, 0.0)])
def test_1080p_preview_sampled(w1080, h1080, theta, d_i, d_r):
    """The benchmark's preview frames.  At 0 deg every low-res pixel centre
    lies on a V_O list edge (1920 / 960 = 2, 1920 / 480 = 4), so every sample
    of a non-empty ray is a tie: those texels are held to the oracle's
    consistent tie resolutions."""
    say(f"[gpu] 1080p preview theta={theta} D_I={d_i} D_R={d_r}")
    check_preview_workload(h1080, w1080, inputs.orbit_camera(theta), 1920, 1080, d_i, d_r, 6000,
                           200 + int(theta), 1000)


@pytest.mark.parametrize("theta", [20.0, 45.0])
def test_1080p_alg_bytes_with_skipping(w1080, h1080, theta):
    """The counts behind the roofline's algorithmic bytes, in the benchmark's
    configuration (skipping on, window search), over whole 1920x1080 frames:
    the supersegments composited equal the oracle's; the lists the walker
    enters lie between those empty-space skipping cannot skip (entered over a
    part of the ray inside a non-empty grid cell) and all lists the rays
    cross, so the bytes lie between the two oracle figures."""
    say(f"[gpu] 1080p counters theta={theta}")
    cam = inputs.orbit_camera(theta)
    img, tl, ts, st = h1080.render_counters(cam, 1920, 1080, ess=True)
    torch.cuda.synchronize()
    ref, ost, otl, ots, ote = oracle.render_exact(w1080, cam, 1920, 1080, stats=True, touched=True, ess=True)
    assert np.abs(img.cpu().numpy() - ref).max() <= TOL
    gl, gs, gst = tl.cpu().numpy().astype(bool), ts.cpu().numpy().astype(bool), st.cpu().numpy()
    otl, ots, ote = otl.astype(bool), ots.astype(bool), ote.astype(bool)
    # FP32 and FP64 early termination may straddle a piece on a few rays.
    assert (gs != ots).sum() <= 2 + 1e-4 * ots.sum()
    assert (ote & ~gl).sum() <= 2 + 1e-4 * ote.sum()
    assert (gl & ~otl).sum() <= 2 + 1e-4 * otl.sum()
    assert np.abs(gst[..., 1] - ost[..., 1]).max() <= 2
    assert (gst[..., 0] >= ost[..., 2] - 2).all() and (gst[..., 0] <= ost[..., 0] + 2).all()
    b_gpu = oracle.b_alg(w1080, gl, gs, 1920 * 1080)
    b_min = oracle.b_alg(w1080, ote, ots, 1920 * 1080)
    b_all = oracle.b_alg(w1080, otl, ots, 1920 * 1080)
    say(f"[gpu]   B_alg: walker {b_gpu / 1e6:.1f} MB, oracle with skipping {b_min / 1e6:.1f} MB, "
        f"without {b_all / 1e6:.1f} MB")
    assert b_min * (1 - 1e-4) <= b_gpu <= b_all * (1 + 1e-4)


@pytest.mark.parametrize("fmt", ["f16", "bf16"])
def test_1080p_precision_forms(w1080, fmt):
    V = _V()
    say(f"[gpu] 1080p precision {fmt}")
    deq = oracle.dequant_f16(w1080.rgba) if fmt == "f16" else oracle.dequant_bf16(w1080.rgba)
    pix = sample_pixels(1920, 1080, 3000, seed=7)
    with V.Vdi(w1080, store=fmt) as h:
        for theta in (0.0, 15.0, 40.0):
            cam = inputs.orbit_camera(theta)
            img = frame(h, cam, 1920, 1080)
            ref_q = oracle.render_exact(w1080, cam, 1920, 1080, pixels=pix, rgba=deq)
            ref_32 = oracle.render_exact(w1080, cam, 1920, 1080, pixels=pix)
            assert np.abs(img[pix] - ref_q).max() <= TOL, theta
            p = psnr(img[pix], ref_32)
            say(f"[gpu] {fmt} theta={theta}: max|d| vs FP32 oracle {np.abs(img[pix] - ref_32).max():.2e}, "
                f"PSNR {p:.1f} dB")
            assert p >= 50.0
