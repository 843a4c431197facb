"""Pins of the FP64 oracle against facts that do not come from the oracle
itself: closed forms, invariants, brute force and special cases.

  c-1  rendering from V_O at the VDI's own resolution reproduces the VDI's own
       composite (each pixel-centre ray stays in its list with l = 1; Sections 4.1, 4.2, Eq. 2)
  c-2  homogeneous slabs between planes of constant V_O depth render to the
       closed-form Beer-Lambert opacity 1 - exp(-sigma L) from any viewpoint
  c-3  opacity in [0, 1], premultiplied colour within [0, A]; removing
       supersegments never lowers transmittance
  c-4  brute-force fine-step marching converges at O(1/M) to the exact result
  and: empty VDI -> 0; mirror symmetry at +-theta; count-grid closed forms;
  preview -> exact as D_R -> 0; upsampling identities; precision rounding.
"""
import math

import numpy as np
import pytest

import inputs
import oracle
from tests import synth


@pytest.fixture(scope="module")
def tiny():
    return inputs.load_workload("tiny")


# ---------------------------------------------------------------- c-1
def test_c1_identity_view_reproduces_own_composite_tiny(tiny):
    out = oracle.render_exact(tiny, tiny.camera, tiny.width, tiny.height)
    ref = synth.composite_at_vo(tiny)
    # The generator's first supersegment starts on the AABB face; its float32
    # front depth can round just outside the box, where the ray is clipped, so
    # l = 1 - O(1e-7) there.
    assert np.abs(out - ref).max() < 1e-6


def test_c1_identity_view_random_vdi():
    v = synth.random_vdi(24, 16, 6, seed=7, zlo=1.05, zhi=1.95)
    out = oracle.render_exact(v, v.camera, v.width, v.height)
    ref = synth.composite_at_vo(v)
    assert np.abs(out - ref).max() < 1e-9


def test_generator_composite_matches_its_dvr(tiny):
    # Compositing inside a supersegment is exact (Section 2.3), so the VDI's own
    # composite equals the generator's DVR up to float32 storage.
    ref = synth.composite_at_vo(tiny)
    assert np.abs(ref - tiny.dvr).max() < 2e-6


# ---------------------------------------------------------------- c-2
def _slab_expected(v, cam, W, H, slabs):
    """Closed form: per pixel ray, world lengths inside each slab and whether
    the crossing lies inside the V_O frustum (computed from the pinhole model)."""
    th = math.tan(math.radians(cam.fov_y_deg) / 2)
    eye = np.array(cam.eye, np.float64)
    F = -eye / np.linalg.norm(eye)
    R = np.cross(F, [0.0, 1.0, 0.0]); R /= np.linalg.norm(R)
    U = np.cross(R, F)
    xs = -1.0 + (2.0 * np.arange(W) + 1.0) / W
    ys = -1.0 + (2.0 * np.arange(H) + 1.0) / H
    X, Y = np.meshgrid(xs, ys)
    d = F[None, None] + (X * th * W / H)[..., None] * R + (Y * th)[..., None] * U
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    eO = np.array(v.camera.eye, np.float64)
    FO = np.array([0.0, 0.0, -1.0])
    thO = math.tan(math.radians(v.camera.fov_y_deg) / 2)
    aO = v.width / v.height
    Zp = d @ FO
    Z0 = (eye - eO) @ FO
    A = np.zeros((H, W)); C = np.zeros((H, W, 3)); T = np.ones((H, W))
    ok = np.ones((H, W), bool)
    for z1, z2, sig, col in slabs:
        z1, z2 = float(np.float32(z1)), float(np.float32(z2))
        for z in (z1, z2):
            t = (z - Z0) / Zp
            P = eye + t[..., None] * d
            rel = P - eO
            xn = rel[..., 0] / (z * thO * aO)
            yn = rel[..., 1] / (z * thO)
            ok &= (np.abs(xn) < 0.999) & (np.abs(yn) < 0.999) & (t > 0)
        a = 1.0 - np.exp(-sig * (z2 - z1) / np.abs(Zp))
        C += (T * a)[..., None] * np.array(col)
        T *= 1.0 - a
    out = np.concatenate([C, (1.0 - T)[..., None]], axis=-1)
    return out, ok


@pytest.mark.parametrize("theta", [0.0, 7.0, 23.0, -31.0])
def test_c2_one_slab_closed_form(theta):
    slabs = [(1.3, 1.55, 3.0, (0.2, 0.6, 0.9))]
    v = synth.slab_vdi(64, 48, slabs)
    cam = inputs.orbit_camera(theta)
    out = oracle.render_exact(v, cam, 40, 30)
    exp, ok = _slab_expected(v, cam, 40, 30, slabs)
    assert ok.sum() > 100
    assert np.abs(out[ok] - exp[ok]).max() < 2e-6


@pytest.mark.parametrize("theta", [4.0, 35.0])
def test_c2_two_slabs_closed_form(theta):
    slabs = [(1.2, 1.4, 2.0, (0.9, 0.1, 0.1)), (1.5, 1.9, 5.0, (0.1, 0.8, 0.3))]
    v = synth.slab_vdi(50, 50, slabs)
    cam = inputs.orbit_camera(theta)
    out = oracle.render_exact(v, cam, 33, 27)
    exp, ok = _slab_expected(v, cam, 33, 27, slabs)
    assert ok.sum() > 100
    assert np.abs(out[ok] - exp[ok]).max() < 2e-6


# ---------------------------------------------------------------- c-3
def test_c3_ranges_and_monotone_transmittance():
    v = synth.random_vdi(20, 14, 5, seed=11)
    cam = inputs.orbit_camera(12.0)
    out = oracle.render_exact(v, cam, 31, 23)
    A = out[..., 3]
    assert A.min() >= 0.0 and A.max() <= 1.0
    assert (out[..., :3] >= -1e-15).all() and (out[..., :3] <= A[..., None] + 1e-12).all()
    # Removing supersegments (dropping the last of every list) never raises opacity
    # by more than the termination threshold.
    w = synth.random_vdi(20, 14, 5, seed=11)
    w.count = np.maximum(w.count.astype(int) - 1, 0).astype(np.uint8)
    out2 = oracle.render_exact(w, cam, 31, 23)
    assert (out2[..., 3] <= A + 1e-5).all()


# ---------------------------------------------------------------- c-4
@pytest.mark.parametrize("seed,theta", [(3, 9.0), (4, 27.0), (5, -15.0)])
def test_c4_bruteforce_converges(seed, theta):
    v = synth.random_vdi(8, 8, 4, seed=seed, alpha_max=0.7, min_thick=0.02)
    cam = inputs.orbit_camera(theta)
    W = H = 12
    pix = np.arange(W * H)
    ex = oracle.render_exact(v, cam, W, H).reshape(-1, 4)
    errs = []
    for M in (2 ** 12, 2 ** 14, 2 ** 16):
        m = oracle.march(v, cam, W, H, pix, M)
        errs.append(np.abs(m - ex).max())
    assert errs[-1] < 2e-3
    assert errs[2] < errs[0] / 4.0  # at least O(1/M) over a 16x refinement, with margin


def test_c4_bruteforce_tiny_workload(tiny):
    cam = inputs.orbit_camera(5.0)
    rng = np.random.default_rng(0)
    pix = rng.choice(tiny.width * tiny.height, 64, replace=False)
    ex = oracle.render_exact(tiny, cam, tiny.width, tiny.height, pixels=pix)
    m = oracle.march(tiny, cam, tiny.width, tiny.height, pix, 2 ** 16)
    assert np.abs(m - ex).max() < 2e-3


# ---------------------------------------------------------------- special cases
def test_empty_vdi_renders_zero():
    v = synth.empty_vdi(16, 16, 4)
    out = oracle.render_exact(v, inputs.orbit_camera(10.0), 20, 20)
    assert not out.any()


def test_mirror_symmetry():
    v = synth.mirror_x(synth.random_vdi(16, 12, 4, seed=21))
    a = oracle.render_exact(v, inputs.orbit_camera(13.0), 18, 14)
    b = oracle.render_exact(v, inputs.orbit_camera(-13.0), 18, 14)
    assert np.abs(a - b[:, ::-1]).max() < 1e-9


def test_backward_and_grazing_rays_are_finite():
    v = synth.random_vdi(16, 12, 4, seed=5)
    for theta in (80.0, 90.0, 100.0, 150.0, 180.0):
        out = oracle.render_exact(v, inputs.orbit_camera(theta), 16, 12)
        assert np.isfinite(out).all() and out[..., 3].max() <= 1.0


def test_ray_from_behind_is_mirror_of_front_for_symmetric_slab():
    # A single slab seen from V_O (theta=0) and from the opposite side (theta=180)
    # through the centre pixel accumulates the same opacity.
    slabs = [(1.3, 1.7, 2.5, (0.5, 0.5, 0.5))]
    v = synth.slab_vdi(9, 9, slabs)
    a = oracle.render_exact(v, inputs.orbit_camera(0.0), 9, 9)[4, 4]
    b = oracle.render_exact(v, inputs.orbit_camera(180.0), 9, 9)[4, 4]
    assert abs(a[3] - b[3]) < 1e-6 and a[3] > 0.5


# ---------------------------------------------------------------- count grid
def test_count_grid_closed_form():
    # Supersegments placed strictly inside known slices.
    v = synth.empty_vdi(20, 12, 3)
    z = v.grid_z.astype(np.float64)
    mid = 0.5 * (z[:-1] + z[1:])
    v.count[:] = 2
    v.depth[0, ..., 0] = mid[2]; v.depth[0, ..., 1] = mid[2] + 1e-4   # inside slice 2
    v.depth[1, ..., 0] = mid[5]; v.depth[1, ..., 1] = mid[7]          # slices 5, 6, 7
    g = oracle.count_grid(v)
    k = v.grid_k
    per_col = np.zeros((2, 3))
    lists = np.array([[min(k, 20 - cx * k) * min(k, 12 - cy * k) for cx in range(3)] for cy in range(2)])
    assert g.shape == (v.grid_nz, 2, 3)
    for c in range(v.grid_nz):
        want = lists * ((c == 2) + (5 <= c <= 7))
        assert (g[c] == want).all(), c
    assert g.sum() == 20 * 12 * 4


def test_count_grid_touching_faces_do_not_count():
    v = synth.empty_vdi(8, 8, 1)
    z = v.grid_z
    v.count[:] = 1
    v.depth[0, ..., 0] = z[3]; v.depth[0, ..., 1] = z[4]   # exactly slice 3
    g = oracle.count_grid(v)
    assert g[3].sum() == 64 and g.sum() == 64


def test_grid_size_matches_paper_full_hd():
    # Section 6.3: the ESS structure of a full-HD VDI is 2.5 MiB; with 8x8
    # lists per cell, 20 depth slices and 4-byte counts it is 2.47 MiB.
    gw, gh = -(-1920 // 8), -(-1080 // 8)
    mib = gw * gh * 20 * 4 / 2 ** 20
    assert round(mib, 1) == 2.5


# ---------------------------------------------------------------- preview
def test_preview_converges_to_exact(tiny):
    cam = inputs.orbit_camera(5.0)
    w = h = 64
    ex = oracle.render_exact(tiny, cam, w, h)
    errs = []
    for dr in (1 / 16, 1 / 256, 1 / 2048):
        pv, fl = oracle.render_preview(tiny, cam, w, h, dr)
        errs.append(np.abs(pv - ex).max())
    assert errs[-1] < 5e-3 and errs[-1] < errs[0]


def test_preview_samples_scale_with_rate(tiny):
    cam = inputs.orbit_camera(5.0)
    # n = ceil(x / D_R) per non-empty cell: for small D_R the total scales as 1/D_R.
    _, _, n1 = oracle.render_preview(tiny, cam, 32, 32, 1 / 32, samples=True)
    _, _, n4 = oracle.render_preview(tiny, cam, 32, 32, 1 / 128, samples=True)
    assert 3.5 < n4.sum() / n1.sum() < 4.05


def test_preview_slab_on_slice_faces_is_exact_from_vo():
    # A slab whose faces are grid slice boundaries: only the cells inside it are
    # non-empty, so every sample lands in the slab, the sample spacings of one
    # ray sum to its length inside the slab, and from V_O itself (one list per
    # ray, l = h / L0 summing to 1) the preview reproduces the stored opacity.
    v = synth.slab_vdi(16, 16, [(1.0, 2.0, 1.0, (0.2, 0.6, 0.9))], half=4.0)
    z = v.grid_z
    assert z[10] > 1.0   # the slab lies in front of V_O's near plane
    v.depth[0, ..., 0] = z[10]
    v.depth[0, ..., 1] = z[14]
    v.rgba[0, ..., 3] = 0.6
    for dr in (0.5, 0.125):
        pv, fl = oracle.render_preview(v, v.camera, 16, 16, dr)
        ex = oracle.render_exact(v, v.camera, 16, 16)
        assert not fl.any()
        assert np.abs(pv[..., 3] - np.float32(0.6)).max() < 1e-9
        assert np.abs(pv - ex).max() < 1e-9


def test_preview_tie_variants_closed_form():
    """Preview rays along list edges (Section 4.4 sampling rule, point
    location on a tie): from V_O at half its resolution every pixel-centre ray
    runs along the edge between list columns 2px and 2px+1 and rows 2py and
    2py+1.  The lists alternate in opacity by column, and the slab's faces are
    grid slice boundaries, so every sample of a ray lies in the slab and a
    ray's exponents h / L0 sum to cos_i / cos_ray.  Resolving the ties
    towards +x (+y) must give list column 2px+1 (row 2py+1) in closed form,
    towards -x (-y) column 2px (row 2py); the unresolved oracle flags them."""
    v = synth.slab_vdi(16, 16, [(1.0, 2.0, 1.0, (0.2, 0.6, 0.9))], half=4.0)
    z = v.grid_z
    v.depth[0, ..., 0] = z[10]
    v.depth[0, ..., 1] = z[14]
    cols = np.arange(16)
    alpha = np.where(cols % 2 == 0, 0.6, 0.3).astype(np.float32)
    rgb = np.where((cols % 2 == 0)[:, None], [[1.0, 0.0, 0.0]], [[0.0, 0.0, 1.0]]).astype(np.float32)
    v.rgba[0, ..., 3] = alpha[None, :]
    v.rgba[0, ..., :3] = rgb[None, :, :]
    cam = v.camera
    pix = np.arange(64)
    _, flags = oracle.render_preview(v, cam, 8, 8, 0.5, pixels=pix)
    assert flags.all()
    var = oracle.preview_tie_variants(v, cam, 8, 8, 0.5, pix)
    th = math.tan(math.radians(cam.fov_y_deg) / 2.0)
    cos_i = synth.list_cos(cam, 16, 16)
    for k, (bx, by, _, _) in enumerate(oracle.TIE_BIASES):
        for q in pix:
            px, py = q % 8, q // 8
            xc, yc = -1.0 + (2 * px + 1) / 8.0, -1.0 + (2 * py + 1) / 8.0
            cos_ray = 1.0 / math.sqrt(1.0 + (xc * th) ** 2 + (yc * th) ** 2)
            col = 2 * px + (1 if bx > 0 else 0)
            row = 2 * py + (1 if by > 0 else 0)
            A = 1.0 - (1.0 - float(alpha[col])) ** (cos_i[row, col] / cos_ray)
            want = np.concatenate([rgb[col] * A, [A]])
            assert np.abs(var[k, q] - want).max() < 1e-9, (k, q)


def test_exact_tie_variants_closed_form():
    """Exact rays along list edges (Sections 4.1-4.2; the field is ambiguous
    on an edge): from V_O at half its resolution every pixel-centre ray runs
    along the corner of list columns 2px, 2px+1 and rows 2py, 2py+1 and stays
    there.  With lists alternating in opacity by column, resolving the ties
    towards +x (+y) must give column 2px+1 (row 2py+1) alone, in closed form
    (Eq. 2 with l = cos_i / cos_ray through the slab), towards -x (-y) column
    2px (row 2py); the unresolved oracle flags every such ray."""
    v = synth.slab_vdi(16, 16, [(1.0, 2.0, 1.0, (0.2, 0.6, 0.9))], half=4.0)
    cols = np.arange(16)
    alpha = np.where(cols % 2 == 0, 0.6, 0.3).astype(np.float32)
    rgb = np.where((cols % 2 == 0)[:, None], [[1.0, 0.0, 0.0]], [[0.0, 0.0, 1.0]]).astype(np.float32)
    v.rgba[0, ..., 3] = alpha[None, :]
    v.rgba[0, ..., :3] = rgb[None, :, :]
    cam = v.camera
    pix = np.arange(64)
    _, flags = oracle.render_exact(v, cam, 8, 8, pixels=pix, flags=True)
    assert flags.all()
    var = oracle.exact_tie_variants(v, cam, 8, 8, pix)
    th = math.tan(math.radians(cam.fov_y_deg) / 2.0)
    cos_i = synth.list_cos(cam, 16, 16)
    for k, (bx, by) in enumerate(oracle.EXACT_TIE_BIASES):
        for q in pix:
            px, py = q % 8, q // 8
            xc, yc = -1.0 + (2 * px + 1) / 8.0, -1.0 + (2 * py + 1) / 8.0
            cos_ray = 1.0 / math.sqrt(1.0 + (xc * th) ** 2 + (yc * th) ** 2)
            col = 2 * px + (1 if bx > 0 else 0)
            row = 2 * py + (1 if by > 0 else 0)
            A = 1.0 - (1.0 - float(alpha[col])) ** (cos_i[row, col] / cos_ray)
            want = np.concatenate([rgb[col] * A, [A]])
            assert np.abs(var[k, q] - want).max() < 1e-9, (k, q)


@pytest.mark.parametrize("theta", [9.0, -31.0])
def test_exact_tie_variants_agree_off_ties(tiny, theta):
    """Off list edges the exact result is unique: no ray of a rotated view at
    an even height is flagged and every resolution gives the unresolved
    result.  At an odd height the middle row lies in V_O's plane y = 0, a
    list-row edge of the 128-row VDI: exactly that row is flagged."""
    cam = inputs.orbit_camera(theta)
    pix = np.arange(48 * 32)
    ref, flags = oracle.render_exact(tiny, cam, 48, 32, pixels=pix, flags=True)
    assert not flags.any()
    var = oracle.exact_tie_variants(tiny, cam, 48, 32, pix)
    assert np.array_equal(var, np.broadcast_to(ref, var.shape))
    img, fl = oracle.render_exact(tiny, cam, 63, 63, flags=True)
    hit = img[..., 3] > 0
    assert not fl[np.arange(63) != 31].any()
    assert fl[31][hit[31]].all()


def test_preview_tie_variants_agree_off_ties(tiny):
    """Resolving ties changes only the results the oracle flags."""
    cam = inputs.orbit_camera(9.0)
    pix = np.arange(48 * 32)
    ref, flags = oracle.render_preview(tiny, cam, 48, 32, 2.0, pixels=pix)
    var = oracle.preview_tie_variants(tiny, cam, 48, 32, 2.0, pix)
    assert (flags == 0).mean() > 0.9
    assert np.array_equal(var[:, flags == 0], np.broadcast_to(ref[flags == 0], var[:, flags == 0].shape))


@pytest.mark.parametrize("theta", [0.0, 20.0, -45.0])
def test_touched_lists_with_skipping_bounds(tiny, theta):
    """The lists that empty-space skipping must still read (entered over a
    part of the ray inside a non-empty grid cell, Section 4.3) lie between
    the lists holding a composited supersegment and all lists entered."""
    cam = inputs.orbit_camera(theta)
    out, st, tl, ts, te = oracle.render_exact(tiny, cam, 96, 80, stats=True, touched=True, ess=True)
    holds = ts.astype(bool).any(axis=0)
    assert (te <= tl).all() and (holds <= te.astype(bool)).all()
    assert (st[..., 2] <= st[..., 0]).all()
    assert te.sum() < tl.sum() and holds.sum() < te.sum()
    assert np.array_equal(out, oracle.render_exact(tiny, cam, 96, 80))
    v = synth.empty_vdi(16, 16, 3)
    _, _, tl0, _, te0 = oracle.render_exact(v, cam, 20, 20, stats=True, touched=True, ess=True)
    assert tl0.sum() > 0 and te0.sum() == 0


def test_upsample_identities():
    rng = np.random.default_rng(1)
    lo = rng.random((7, 9, 4))
    same, _ = oracle.upsample(lo, 9, 7)
    assert np.abs(same - lo).max() < 1e-15
    const, _ = oracle.upsample(np.full((5, 6, 4), 0.37), 17, 11)
    assert np.abs(const - 0.37).max() < 1e-15
    # A linear ramp in x is reproduced exactly away from the clamped border.
    xs = np.arange(8, dtype=np.float64)
    ramp = np.broadcast_to((2.0 * xs + 1.0)[None, :, None], (4, 8, 4)).copy()
    up, _ = oracle.upsample(ramp, 16, 8)
    X = np.arange(16)
    want = 2.0 * ((X + 0.5) / 2.0 - 0.5) + 1.0
    inner = slice(1, 15)
    assert np.abs(up[:, inner, 0] - want[inner]).max() < 1e-12


def test_full_render_di1_dr0_is_exact(tiny):
    cam = inputs.orbit_camera(5.0)
    a, fl = oracle.render(tiny, cam, 40, 30, 1.0, 0.0)
    b = oracle.render_exact(tiny, cam, 40, 30)
    assert np.array_equal(a, b) and not fl.any()


@pytest.mark.parametrize("d_i", [2.0, 3.0, 4.0])
@pytest.mark.parametrize("d_r", [0.0, 2.0])
def test_render_points_equals_full_render(tiny, d_i, d_r):
    """The sampled-pixel form used for large frames (each output pixel's four
    low-res texels rendered one by one, then combined bilinearly) equals the
    whole-frame render followed by the upsampling pass, flags included."""
    cam = inputs.orbit_camera(11.0)
    W, H = 128, 96
    full, fl = oracle.render(tiny, cam, W, H, d_i, d_r)
    pix = np.random.default_rng(int(d_i * 10 + d_r)).choice(W * H, 2000, replace=False)
    pix = np.concatenate([pix, [0, W - 1, (H - 1) * W, W * H - 1]])
    pts, pfl = oracle.render_points(tiny, cam, W, H, d_i, d_r, pix)
    assert np.abs(pts - full.reshape(-1, 4)[pix]).max() < 1e-12
    assert np.array_equal(pfl, fl.reshape(-1)[pix])
    assert (full[..., 3] > 0).mean() > 0.2


def test_lowres_size():
    assert oracle.lowres_size(1920, 1080, 2.0) == (960, 540)
    assert oracle.lowres_size(1920, 1080, 4.0) == (480, 270)
    assert oracle.lowres_size(5, 3, 100.0) == (1, 1)
    assert oracle.lowres_size(1280, 720, 3.0) == (427, 240)


# ---------------------------------------------------------------- precision
def test_bf16_rounding_known_values():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -8 + 2 ** -20, 0.1, -2.5, 0.0],
                    dtype=np.float32)
    got = oracle.dequant_bf16(vals)
    # ties go to the even mantissa; above-tie rounds up; exact values stay
    want = np.array([1.0, 1.0, 1.0 + 4 * 2 ** -8, 1.0 + 2 * 2 ** -8, 0.10009765625, -2.5, 0.0], dtype=np.float32)
    assert np.array_equal(got, want)


def test_f16_rounding_known_values():
    vals = np.array([1.0, 1.0 + 2 ** -11, 1.0 + 3 * 2 ** -11, 0.1, 65504.0, 2 ** -24], dtype=np.float32)
    got = oracle.dequant_f16(vals)
    want = np.array([1.0, 1.0, 1.0 + 2 * 2 ** -10, 0.0999755859375, 65504.0, 2 ** -24], dtype=np.float32)
    assert np.array_equal(got, want)
