"""vdi_render_batch through the C ABI (needs an MI355X): every frame of a
batch is bit-identical to the same vdi_render, and matches the FP64 oracle
(fed the stored, rounded colours); frames of several VDIs and colour formats,
ragged sizes, exact and preview modes in one call; the largest batch; many
calls in a row on one stream (the pinned job-table ring); argument errors
launch nothing."""
import sys

import numpy as np
import pytest

import inputs
import oracle
from tests.gpu_util import oracle_check

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


@pytest.fixture(scope="module")
def sources():
    return [inputs.load_workload("tiny"), inputs.load_workload("720p", keep_dvr=False)]


@pytest.fixture(scope="module")
def handles(sources):
    from paper_2206_08660_amd import vdi as V
    hs = [V.Vdi(sources[0]), V.Vdi(sources[1], store="f16"), V.Vdi(sources[0], store="bf16")]
    yield hs
    for h in hs:
        h.close()


MODES = [(1.0, 0.0), (2.0, 2.0), (1.0, 0.5), (3.0, 1.0), (4.0, 2.0)]
SIZES = [(128, 128), (97, 61), (1280, 720), (640, 360), (33, 200)]


def frames_mix(handles, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        hi = int(rng.integers(0, 3))
        W, H = SIZES[int(rng.integers(0, len(SIZES)))] if hi == 1 else SIZES[[0, 1, 4][int(rng.integers(0, 3))]]
        di, dr = MODES[int(rng.integers(0, len(MODES)))]
        out.append((hi, float(rng.uniform(-40, 40)), W, H, di, dr))
    return out


def run_batch(handles, spec, stream=None):
    from paper_2206_08660_amd import vdi as V
    outs = [torch.full((H, W, 4), -1.0, dtype=torch.float32, device="cuda") for (_, _, W, H, _, _) in spec]
    V.render_batch([(handles[hi], inputs.orbit_camera(yaw), W, H, di, dr, o)
                    for (hi, yaw, W, H, di, dr), o in zip(spec, outs)], stream=stream)
    return outs


def test_batch_matches_single_renders_and_the_oracle(sources, handles):
    spec = frames_mix(handles, 40, seed=5)
    assert len({s[0] for s in spec}) == 3 and len({s[4:] for s in spec}) == len(MODES)
    outs = run_batch(handles, spec)
    torch.cuda.synchronize()
    for (hi, yaw, W, H, di, dr), o in zip(spec, outs):
        alone = handles[hi].render(inputs.orbit_camera(yaw), W, H, di, dr)
        torch.cuda.synchronize()
        a, b = alone.cpu().numpy(), o.cpu().numpy()
        assert np.array_equal(a, b), (hi, yaw, W, H, di, dr, np.abs(a - b).max())
    # The largest frame of every (VDI, mode) pair that occurs, against the
    # oracle on the colours the VDI stores.  Downsampled previews of small
    # frames have few low-res texels, each read by many output pixels, so
    # fewer of their pixels avoid every tie; at least 30% must, and a minimum
    # of non-empty pixels is compared.
    rgba = [None, oracle.dequant_f16(sources[1].rgba), oracle.dequant_bf16(sources[0].rgba)]
    src = [sources[0], sources[1], sources[0]]
    largest = {}
    for i, (hi, yaw, W, H, di, dr) in enumerate(spec):
        key = (hi, di, dr)
        if key not in largest or W * H > spec[largest[key]][2] * spec[largest[key]][3]:
            largest[key] = i
    for key, i in sorted(largest.items()):
        hi, yaw, W, H, di, dr = spec[i]
        say(f"[gpu] batch frame {i} vs oracle: VDI {hi}, yaw {yaw:.1f}, {W}x{H}, D_I={di}, D_R={dr}")
        ne = oracle_check(src[hi], rgba[hi], inputs.orbit_camera(yaw), W, H, di, dr, outs[i].cpu().numpy(), seed=i,
                          min_ok=0.3)
        assert ne >= (20 if hi != 1 else 200), ne
    assert len(largest) >= 10


def test_largest_batch_and_many_calls_in_a_row(handles):
    """VDI_BATCH_MAX_FRAMES small frames in one call; then ten calls queued on
    one stream without waiting (more than the four pinned job-table slots),
    each frame equal to its vdi_render."""
    from paper_2206_08660_amd import vdi as V
    n = 1024
    rng = np.random.default_rng(11)
    spec = [(int(rng.integers(0, 3)), float(rng.uniform(-60, 60)), 24 + int(rng.integers(0, 9)),
             16 + int(rng.integers(0, 9)), *MODES[int(rng.integers(0, len(MODES)))]) for _ in range(n)]
    outs = run_batch(handles, spec)
    torch.cuda.synchronize()
    for k in range(0, n, 37):
        hi, yaw, W, H, di, dr = spec[k]
        a = handles[hi].render(inputs.orbit_camera(yaw), W, H, di, dr).cpu().numpy()
        assert np.array_equal(a, outs[k].cpu().numpy()), k
    calls = [frames_mix(handles, 6, seed=100 + c) for c in range(10)]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        results = [run_batch(handles, spec_c, stream=s) for spec_c in calls]
    s.synchronize()
    for spec_c, outs_c in zip(calls, results):
        for (hi, yaw, W, H, di, dr), o in zip(spec_c, outs_c):
            a = handles[hi].render(inputs.orbit_camera(yaw), W, H, di, dr).cpu().numpy()
            assert np.array_equal(a, o.cpu().numpy()), (hi, yaw, W, H, di, dr)
    with pytest.raises(V.VdiError):
        V.render_batch([(handles[0], inputs.orbit_camera(0.0), 8, 8, 1.0, 0.0,
                         torch.empty((8, 8, 4), dtype=torch.float32, device="cuda"))] * (n + 1))


def test_errors_launch_nothing(handles):
    """A bad frame anywhere in the batch: the call fails with VDI_ERR_ARG,
    naming the frame, and no output is written."""
    from paper_2206_08660_amd import vdi as V
    spec = frames_mix(handles, 6, seed=7)
    outs = [torch.full((H, W, 4), -1.0, dtype=torch.float32, device="cuda") for (_, _, W, H, _, _) in spec]
    frames = [(handles[hi], inputs.orbit_camera(yaw), W, H, di, dr, o) for (hi, yaw, W, H, di, dr), o in zip(spec, outs)]
    hi, yaw, W, H, di, dr = spec[4]
    bad = list(frames)
    bad[4] = (handles[hi], inputs.orbit_camera(yaw), W, H, 0.5, dr, outs[4])   # D_I < 1
    with pytest.raises(V.VdiError) as ei:
        V.render_batch(bad)
    assert ei.value.code == V.VDI_ERR_ARG and "frame 4" in str(ei.value)
    bad[4] = (handles[hi], inputs.orbit_camera(yaw), W, H, di, 5e-5, outs[4])  # 0 < D_R < 1e-4
    with pytest.raises(V.VdiError):
        V.render_batch(bad)
    torch.cuda.synchronize()
    assert all(bool((o == -1.0).all()) for o in outs)
    V.render_batch(frames)
    torch.cuda.synchronize()
    assert not any(bool((o == -1.0).all()) for o in outs)
