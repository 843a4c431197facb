"""Pins of the seeded VDI generator (paper Section 3, Eq. 1, supplement Alg. S1).

The generator is the input producer for both the oracle and the HIP library;
these tests check its output against facts it must satisfy by construction."""
import math

import numpy as np
import pytest

import inputs
from tests import slabs


def _structure_ok(v: inputs.VDI):
    n = v.count.astype(int)
    assert n.max() <= v.ns
    for j in range(v.ns):
        valid = n > j
        f, b = v.depth[j, ..., 0], v.depth[j, ..., 1]
        assert (b[valid] > f[valid]).all()
        assert not v.depth[j][~valid].any() and not v.rgba[j][~valid].any()
        a = v.rgba[j, ..., 3][valid]
        assert (a > 0).all() and (a <= 1).all()
        c = v.rgba[j, ..., :3][valid]
        assert (c >= -1e-6).all() and (c <= 1 + 1e-6).all()
        if j + 1 < v.ns:
            nxt = n > j + 1
            assert (v.depth[j + 1, ..., 0][nxt] >= b[nxt]).all()   # sorted, non-overlapping


@pytest.fixture(scope="module")
def tiny():
    return inputs.load_workload("tiny")


@pytest.fixture(scope="module")
def w720():
    return inputs.load_workload("720p")


def test_tiny_structure(tiny):
    _structure_ok(tiny)
    assert tiny.count.max() >= 3 and (tiny.count > 0).mean() > 0.3


def test_720p_structure_and_bisection(w720):
    v = w720
    _structure_ok(v)
    ns, delta = v.ns, int(math.floor(0.15 * v.ns))
    hit = v.count > 0
    g, nu = v.gamma[hit], v.nuncapped[hit]
    first = g == 1e-5
    # Rays accepted at the initial gamma produce at most N_S; every other ray
    # ends inside the tolerance band or with the bracket collapsed.
    assert (nu[first] <= ns).all()
    band = (nu >= ns - delta) & (nu <= ns)
    assert (band | first).mean() > 0.99
    assert (nu[~first] <= ns).mean() > 0.99


def _ramp_volume(n=32):
    # A block whose value rises along z, so consecutive samples all differ.
    vol = np.zeros((n, n, n), np.float32)
    for k in range(8, 24):
        vol[k, 8:24, 8:24] = 0.2 + 0.6 * (k - 8) / 15.0
    return vol


def _samples_above(vol, cam, w, h, px, py, thresh):
    """Count the generator's midpoint samples whose trilinear value exceeds
    `thresh` on the ray of pixel (px, py) (equal-length partition of the
    AABB-clipped ray, one voxel of the longest axis at most)."""
    n = vol.shape[0]
    th = math.tan(math.radians(cam.fov_y_deg) / 2)
    eye = np.array(cam.eye, np.float64)
    d = np.array([(-1 + (2 * px + 1) / w) * th * w / h, (-1 + (2 * py + 1) / h) * th, -1.0])
    d /= np.linalg.norm(d)
    ts = []
    for a in range(3):
        if abs(d[a]) > 1e-12:
            ta, tb = (-0.5 - eye[a]) / d[a], (0.5 - eye[a]) / d[a]
            ts.append((min(ta, tb), max(ta, tb)))
    t0 = max(x[0] for x in ts)
    t1 = min(x[1] for x in ts)
    N = int(math.ceil((t1 - t0) * n - 1e-9))
    L = (t1 - t0) / N
    cnt = 0
    for q in range(N):
        P = eye + (t0 + (q + 0.5) * L) * d
        u = (P + 0.5) * n - 0.5
        i0 = np.floor(u).astype(int)
        w_ = u - i0
        val = 0.0
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    ii = np.clip(i0 + [dx, dy, dz], 0, n - 1)
                    wt = (w_[0] if dx else 1 - w_[0]) * (w_[1] if dy else 1 - w_[1]) * (w_[2] if dz else 1 - w_[2])
                    val += wt * vol[ii[2], ii[1], ii[0]]
        cnt += val > thresh
    return cnt


def test_gamma_extremes_on_ramp():
    vol = _ramp_volume()
    cam = inputs.orbit_camera(0.0)
    w = h = 16
    big = inputs.generate_vdi(vol, cam, w, h, 255, inputs.TF_RAMP, gamma=10.0)      # gamma > sqrt(3)
    small = inputs.generate_vdi(vol, cam, w, h, 255, inputs.TF_RAMP, gamma=1e-12)   # gamma -> 0+
    hit = big.count > 0
    assert hit.sum() > 20
    assert (big.count[hit] == 1).all()               # one supersegment per non-transparent run
    for (px, py) in [(7, 7), (8, 8), (6, 9)]:
        want = _samples_above(vol, cam, w, h, px, py, 0.05)   # ramp TF is transparent at v <= 0.05
        assert want > 5
        assert small.count[py, px] == want              # one supersegment per non-transparent sample
    capped = inputs.generate_vdi(vol, cam, w, h, 4, inputs.TF_RAMP, gamma=1e-12)
    assert (capped.count[hit] == np.minimum(small.count[hit], 4)).all()
    # The capped list's last supersegment absorbs everything behind it ("smearing").
    py, px = 8, 8
    assert capped.depth[3, py, px, 1] == small.depth[small.count[py, px] - 1, py, px, 1]


def test_homogeneous_block_never_splits():
    n = 32
    vol = np.zeros((n, n, n), np.float32)
    vol[8:24, 8:24, 8:24] = 0.6
    cam = inputs.orbit_camera(0.0)
    v = inputs.generate_vdi(vol, cam, 16, 16, 16, inputs.TF_RAMP, gamma=1e-3)
    # Interior rays see a constant value between two interpolation ramps; the
    # constant run must merge into one supersegment (Eq. 1 distance 0).
    c = v.count[6:10, 6:10]
    assert c.max() <= 5 and c.min() >= 1
    assert v.count.sum() < 16 * 16 * 5


def test_seeded_volumes_are_deterministic():
    a = inputs.volume_blobs(1001)
    b = inputs.volume_blobs(1001)
    c = inputs.volume_blobs(1002)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    s1 = inputs.volume_slab_u16(7, (32, 32, 32))
    s2 = inputs.volume_slab_u16(7, (32, 32, 32))
    assert np.array_equal(s1, s2) and s1.max() > 0


def test_vdi_byte_sizes_match_paper():
    # Section 6.3: 422 MiB (1280x720) and 950 MiB (1920x1080) uncompressed with
    # N_S = 20; Section 6.1: 480 MB at 1024x1024.  RGBA32F + two R32F depths.
    sizes = {(1280, 720): 422, (1920, 1080): 950, (1024, 1024): 480}
    for (w, h), mib in sizes.items():
        v = inputs.VDI(width=w, height=h, ns=20, camera=inputs.orbit_camera(0), bmin=(0,) * 3, bmax=(1,) * 3,
                       count=np.zeros((1, 1), np.uint8), depth=np.zeros((1,), np.float32),
                       rgba=np.zeros((1,), np.float32), grid_z=np.zeros(21, np.float32))
        assert abs(v.nbytes_fp32 / 2 ** 20 - mib) < 1.0   # the paper rounds (949.2 -> "950")


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("side", [-1, 1])
def test_eq1_two_layers_closed_form(side):
    """Eq. 1 at an intermediate gamma: the centre ray meets 16 samples of
    v = 0.8 then 16 of v = 0.3; their distance d = |c1 a1 - c2 a2| = 0.1375 is
    the only one that can split it.  Just below d: two supersegments, each
    layer's own colour and opacity 1 - (1 - a)^16, faces at depths 1.0, 1.5,
    2.0; just above: one, their front-to-back merge."""
    runs = slabs.run(slabs.TWO)
    d = slabs.eq1_distance(runs[:1], slabs.TWO[1][0])
    assert abs(d - 0.13747) < 1e-4
    g = d * (1.0 + side * 1e-6)
    v = inputs.generate_vdi(slabs.volume(slabs.TWO), slabs.camera(), slabs.W, slabs.H, 4, inputs.TF_RAMP, gamma=g)
    want = slabs.expected(slabs.TWO, g, 4)
    assert len(want) == (2 if side < 0 else 1)
    slabs.check(v.count, v.depth, v.rgba, want)


@pytest.mark.parametrize("gamma,n", slabs.THREE_CASES)
def test_eq1_three_layers_normalised_open_supersegment(gamma, n):
    """With three layers the distance to the third depends on what the open
    supersegment holds: the second layer alone (0.0591) or the first two
    merged (0.1126, their opacity normalised to one sample length, the
    reading under which a constant run never splits).  Counts 3, 2, 2, 1 at
    gamma 0.05, 0.08, 0.105, 0.2, with the closed-form faces and colours."""
    v = inputs.generate_vdi(slabs.volume(slabs.THREE), slabs.camera(), slabs.W, slabs.H, 8, inputs.TF_RAMP,
                            gamma=gamma)
    want = slabs.expected(slabs.THREE, gamma, 8)
    assert len(want) == n
    slabs.check(v.count, v.depth, v.rgba, want)


def test_gamma_search_end_states_closed_form():
    """The bracket search (supplement Alg. S1) on layered rays: with two
    layers and N_S = 2 the first trial (1e-5, two supersegments) stands; with
    N_S = 1 it gives too many, and the first midpoint (1e-5 + sqrt 3) / 2,
    above d, gives one and stands.  With three layers and N_S = 2 the fourth
    midpoint stands (searched_gamma_three)."""
    cam = slabs.camera()
    v2 = inputs.generate_vdi(slabs.volume(slabs.TWO), cam, slabs.W, slabs.H, 2, inputs.TF_RAMP, gamma=0.0)
    assert v2.gamma[slabs.CY, slabs.CX] == 1e-5 and v2.count[slabs.CY, slabs.CX] == 2
    v1 = inputs.generate_vdi(slabs.volume(slabs.TWO), cam, slabs.W, slabs.H, 1, inputs.TF_RAMP, gamma=0.0)
    assert abs(v1.gamma[slabs.CY, slabs.CX] - 0.5 * (1e-5 + math.sqrt(3.0))) < 1e-12
    slabs.check(v1.count, v1.depth, v1.rgba, slabs.expected(slabs.TWO, 1.0, 1))
    v3 = inputs.generate_vdi(slabs.volume(slabs.THREE), cam, slabs.W, slabs.H, 2, inputs.TF_RAMP, gamma=0.0)
    g = v3.gamma[slabs.CY, slabs.CX]
    assert abs(g - slabs.searched_gamma_three()) < 1e-12
    slabs.check(v3.count, v3.depth, v3.rgba, slabs.expected(slabs.THREE, g, 2))
