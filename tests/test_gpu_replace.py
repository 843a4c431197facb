"""Double-buffered VDI replacement through the C ABI (needs an MI355X): a new
VDI (another generating view, same shape) is uploaded while the old one is
rendered, and swapped in only when complete.  Renders before the swap are
the old VDI's, renders after it are bit-identical to a fresh vdi_create of
the new one."""
import sys
import threading
import time

import numpy as np
import pytest

import inputs
import oracle
from tests.gpu_util import TOL, nonempty_stratum, sample_pixels

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


def _render(h, cam, W, H, **kw):
    img = h.render(cam, W, H, **kw)
    torch.cuda.synchronize()
    return img.cpu().numpy()


def _wait_swap(h, timeout=20.0):
    t0 = time.time()
    while not h.replace_poll():
        assert time.time() - t0 < timeout, "replacement did not complete"
        time.sleep(0.001)


def test_replace_swaps_only_when_complete():
    from paper_2206_08660_amd import vdi as V
    a = inputs.load_workload("tiny")
    b = inputs.load_workload("tiny", base_deg=40.0)
    cam = inputs.orbit_camera(12.0)
    with V.Vdi(b) as hb:
        want_b = _render(hb, cam, 96, 80)
        want_b_prev = _render(hb, cam, 96, 80, d_i=2.0, d_r=1.0)
        grid_b = hb.grid()
    with V.Vdi(a) as h:
        want_a = _render(h, cam, 96, 80)
        assert not h.replace_poll()            # nothing pending
        h.replace_begin(b)
        # The current VDI is still a until a poll swaps.
        assert np.array_equal(_render(h, cam, 96, 80), want_a)
        _wait_swap(h)
        assert not h.replace_poll()
        after = _render(h, cam, 96, 80)
        after_prev = _render(h, cam, 96, 80, d_i=2.0, d_r=1.0)
        assert np.array_equal(after, want_b)
        assert np.array_equal(after_prev, want_b_prev)
        assert np.array_equal(h.grid(), grid_b)
        # The swapped-in VDI renders as the oracle renders b (Section 5: the
        # client renders the newest VDI it holds).
        assert np.abs(after - oracle.render_exact(b, cam, 96, 80)).max() <= TOL
        ref, flags = oracle.render(b, cam, 96, 80, 2.0, 1.0)
        ok = flags == 0
        assert ok.mean() > 0.9 and (ok & (ref[..., 3] > 0)).sum() >= 1000
        assert np.abs(after_prev - ref)[ok].max() <= TOL
        # Back to a: the second replacement writes into the buffers a used before.
        h.replace_begin(a)
        _wait_swap(h)
        assert np.array_equal(_render(h, cam, 96, 80), want_a)
        assert h.info().device_bytes > 0


def test_replace_rejects_other_shapes_and_a_second_pending_one():
    from paper_2206_08660_amd import vdi as V
    a = inputs.load_workload("tiny")
    other = inputs.load_workload("720p", keep_dvr=False)
    with V.Vdi(a) as h:
        with pytest.raises(V.VdiError) as e:
            h.replace_begin(other)
        assert e.value.code == V.VDI_ERR_ARG
        with pytest.raises(V.VdiError) as e:
            h.replace_begin(a, rgba_in=a.rgba.astype(np.float16), fmt_in="f16")
        assert e.value.code == V.VDI_ERR_ARG   # 16-bit input into a float32 VDI
        h.replace_begin(a)
        with pytest.raises(V.VdiError) as e:
            h.replace_begin(a)
        assert e.value.code == V.VDI_ERR_STATE
        _wait_swap(h)


def test_rendering_continues_during_replacement():
    """720p: a second thread replaces the VDI while the main thread keeps
    rendering on one stream; every frame is exactly the old or the new image."""
    from paper_2206_08660_amd import vdi as V
    a = inputs.load_workload("720p", keep_dvr=False)
    b = inputs.load_workload("720p", base_deg=90.0, keep_dvr=False)
    cam = inputs.orbit_camera(20.0)
    W, H = 640, 360
    with V.Vdi(b) as hb:
        want_b = _render(hb, cam, W, H)
    with V.Vdi(a) as h:
        want_a = _render(h, cam, W, H)
        stream = torch.cuda.current_stream()
        err = []

        def replace():
            try:
                h.replace_begin(b, stream=stream)
            except Exception as ex:   # reported by the main thread
                err.append(ex)

        th = threading.Thread(target=replace)
        th.start()
        frames, swapped_at = [], None
        t0 = time.time()
        while swapped_at is None:
            assert time.time() - t0 < 30.0, "replacement did not complete"
            frames.append(_render(h, cam, W, H))
            if not th.is_alive() and h.replace_poll():
                swapped_at = len(frames)
        th.join()
        assert not err, err
        frames.append(_render(h, cam, W, H))
        say(f"[gpu] {swapped_at} frames rendered from the old VDI during the replacement")
        for k, img in enumerate(frames):
            want = want_a if k < swapped_at else want_b
            assert np.array_equal(img, want), k
        assert swapped_at >= 1
    # The last frame, from the swapped-in VDI, against the oracle on b.
    last = frames[-1].reshape(-1, 4).astype(np.float64)
    pix = np.unique(np.concatenate([sample_pixels(W, H, 3000, seed=5), nonempty_stratum(frames[-1], 1500, seed=5)]))
    ref = oracle.render_exact(b, cam, W, H, pixels=pix)
    assert np.abs(last[pix] - ref).max() <= TOL
    assert (ref[:, 3] > 0).sum() >= 1000
