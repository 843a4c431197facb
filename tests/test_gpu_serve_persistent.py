"""Served form with one persistent kernel (vdi_server_create_persistent,
needs an MI355X): each request's image is the same alone (vdi_render) and
in the mix, and matches the FP64 oracle (fed the stored, rounded colours);
admission by budget and slots; the launch ends and a new one starts when a
request of another colour format arrives, when a VDI is created, and after
the server idles."""
import sys
import time

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
    hs = [V.Vdi(sources[0], store="f16"), V.Vdi(sources[1], store="f16"), V.Vdi(sources[0])]
    yield hs
    for h in hs:
        h.close()


def _mix(n, seed, vdis):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        hi = vdis[i % len(vdis)]
        big = hi == 1
        W, H = [(128, 128), (96, 64), (1280, 720), (640, 360)][(i // 8) % 4] if big else [(128, 128), (70, 44)][(i // 8) % 2]
        di, dr = [(1.0, 0.0), (2.0, 2.0), (1.0, 0.5), (4.0, 2.0)][(i // 2) % 4]
        reqs.append((hi, float(rng.uniform(-30, 30)), W, H, di, dr))
    return reqs


def _serve(handles, reqs, **kw):
    from paper_2206_08660_amd import serve
    outs = [torch.full((H, W, 4), -1.0, dtype=torch.float32, device="cuda") for (_, _, W, H, _, _) in reqs]
    torch.cuda.synchronize()
    with serve.Server(8 * 2 ** 30, max_inflight=128, persistent=True, **kw) as srv:
        tickets = []
        for (hi, yaw, W, H, di, dr), buf in zip(reqs, outs):
            t = srv.submit(handles[hi], inputs.orbit_camera(yaw), W, H, di, dr, buf)
            assert t is not None
            tickets.append(t)
        srv.drain()
        assert all(srv.poll(t) for t in tickets)
        st = srv.stats()
    return outs, st


def _same_as_single(handles, reqs, outs):
    for (hi, yaw, W, H, di, dr), buf in zip(reqs, outs):
        alone = handles[hi].render(inputs.orbit_camera(yaw), W, H, di, dr)
        torch.cuda.synchronize()
        a, b = alone.cpu().numpy(), buf.cpu().numpy()
        assert np.array_equal(a, b), (hi, yaw, W, H, di, dr, np.abs(a - b).max())


def test_one_launch_serves_the_mix(sources, handles):
    """96 requests over two FP16 VDIs, every mode and size of the mix,
    submitted back to back: one launch renders them all; every image equals
    its single render, and one of each mode on each VDI matches the oracle."""
    reqs = _mix(96, 5, (0, 1))
    outs, st = _serve(handles, reqs)
    say(f"[gpu] persistent: {st['completed']} requests in {st['batches']} launch(es), peak in flight "
        f"{st['peak_inflight']}")
    assert st["completed"] == len(reqs) and st["inflight"] == 0 and st["queued"] == 0
    assert st["batches"] == 1 and st["peak_inflight"] > 1
    _same_as_single(handles, reqs, outs)
    rgba = [oracle.dequant_f16(sources[0].rgba), oracle.dequant_f16(sources[1].rgba)]
    checked = [0, 2, 4, 6, 17, 19, 21, 23]
    assert len({reqs[i][0:1] + reqs[i][4:] for i in checked}) == 8
    for i in checked:
        hi, yaw, W, H, di, dr = reqs[i]
        say(f"[gpu] persistent request {i} vs oracle: VDI {hi}, yaw {yaw:.1f}, {W}x{H}, D_I={di}, D_R={dr}")
        ne = oracle_check(sources[hi % 2], rgba[hi], inputs.orbit_camera(yaw), W, H, di, dr, outs[i].cpu().numpy(),
                          seed=i)
        assert ne >= (100 if hi == 0 else 1000), ne


def test_colour_formats_alternate(sources, handles):
    """Requests alternating between an FP32 and an FP16 VDI: a launch serves
    one format, so each change of format ends the launch and starts another;
    images equal their single renders, the FP32 ones match the oracle."""
    reqs = _mix(24, 6, (2, 1))
    outs, st = _serve(handles, reqs, waves_per_simd=4)
    say(f"[gpu] persistent, alternating formats: {st['completed']} requests in {st['batches']} launches")
    assert st["completed"] == len(reqs) and st["batches"] >= 12
    _same_as_single(handles, reqs, outs)
    for i in (0, 4):
        hi, yaw, W, H, di, dr = reqs[i]
        assert hi == 2
        ne = oracle_check(sources[0], None, inputs.orbit_camera(yaw), W, H, di, dr, outs[i].cpu().numpy(), seed=i)
        assert ne >= 100, ne


def test_admission_by_budget_and_slots(handles):
    """Budget and slots as in the batched server: a long request in flight
    (a D_R = 0.01 preview of the 720p VDI at 40 deg, tens of ms) makes a
    second one that does not fit be rejected; once it is done, it fits."""
    from paper_2206_08660_amd import serve
    one = 1280 * 720 * 16
    with serve.Server(one + one // 2, max_inflight=8, persistent=True) as srv:
        bufs = [torch.empty((720, 1280, 4), dtype=torch.float32, device="cuda") for _ in range(2)]
        torch.cuda.synchronize()
        t1 = srv.submit(handles[1], inputs.orbit_camera(40.0), 1280, 720, 1.0, 0.01, bufs[0])
        assert t1 is not None
        t2 = srv.submit(handles[1], inputs.orbit_camera(10.0), 1280, 720, 1.0, 0.0, bufs[1])
        assert t2 is None and not srv.poll(t1)
        st = srv.stats()
        assert st["rejected_budget"] == 1 and st["inflight"] == 1 and st["bytes_in_flight"] == one
        srv.drain()
        t2 = srv.submit(handles[1], inputs.orbit_camera(10.0), 1280, 720, 1.0, 0.0, bufs[1])
        assert t2 is not None
        srv.drain()
        assert srv.poll(t1) and srv.poll(t2) and srv.stats()["completed"] == 2
    with serve.Server(2 ** 34, max_inflight=1, persistent=True) as srv:
        b = [torch.empty((720, 1280, 4), dtype=torch.float32, device="cuda"),
             torch.empty((128, 128, 4), dtype=torch.float32, device="cuda")]
        torch.cuda.synchronize()
        t = srv.submit(handles[1], inputs.orbit_camera(40.0), 1280, 720, 1.0, 0.01, b[0])
        assert t is not None
        assert srv.submit(handles[0], inputs.orbit_camera(5.0), 128, 128, 1.0, 0.0, b[1]) is None
        assert srv.stats()["rejected_slots"] == 1
        srv.drain()
        assert srv.poll(t)
    single = handles[1].render(inputs.orbit_camera(40.0), 1280, 720, 1.0, 0.01)
    torch.cuda.synchronize()
    assert torch.equal(single, b[0])


def test_new_vdi_and_idle_restart(sources, handles):
    """A VDI created while a launch is resident: its requests go to a new
    launch, which reads it afresh.  After the server idles (20 ms) the launch
    ends, the device is free for other work, and the next request starts a
    new launch."""
    from paper_2206_08660_amd import serve
    from paper_2206_08660_amd import vdi as V
    cam = inputs.orbit_camera(12.0)
    with serve.Server(2 ** 34, max_inflight=16, persistent=True) as srv:
        a = torch.empty((128, 128, 4), dtype=torch.float32, device="cuda")
        b = torch.empty((128, 128, 4), dtype=torch.float32, device="cuda")
        c = torch.empty((128, 128, 4), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        t = srv.submit(handles[0], cam, 128, 128, 1.0, 0.0, a)
        srv.drain()
        assert srv.poll(t) and srv.stats()["batches"] == 1
        h = V.Vdi(sources[0], store="f16")   # created while the launch is resident
        t = srv.submit(h, inputs.orbit_camera(-7.0), 128, 128, 2.0, 2.0, b)
        srv.drain()
        assert srv.poll(t) and srv.stats()["batches"] == 2
        time.sleep(0.1)                       # the launch idles out
        side = torch.cuda.Stream()
        t0 = time.perf_counter()
        with torch.cuda.stream(side):
            img = handles[0].render(cam, 128, 128, stream=side)
        side.synchronize()
        say(f"[gpu] render beside an idle persistent server: {(time.perf_counter() - t0) * 1e3:.2f} ms")
        assert torch.equal(img, a)
        t = srv.submit(handles[0], cam, 128, 128, 1.0, 0.0, c)
        srv.drain()
        assert srv.poll(t) and srv.stats()["batches"] == 3
        assert torch.equal(c, a)
    alone = h.render(inputs.orbit_camera(-7.0), 128, 128, 2.0, 2.0)
    torch.cuda.synchronize()
    assert torch.equal(alone, b)
    h.close()
    rgba = oracle.dequant_f16(sources[0].rgba)
    ne = oracle_check(sources[0], rgba, cam, 128, 128, 1.0, 0.0, a.cpu().numpy(), seed=1)
    assert ne >= 100, ne


def test_replacement_swap_starts_a_new_launch(sources):
    """A VDI (BF16 colour) replaced while a launch is resident: the request
    before the swap renders the old VDI, the one after it the new VDI,
    bit-identical to a fresh vdi_create of it, in a new launch (the launch
    reads VDIs through caches nothing invalidates while it runs)."""
    from paper_2206_08660_amd import serve
    from paper_2206_08660_amd import vdi as V
    b = inputs.load_workload("tiny", base_deg=40.0)
    cam = inputs.orbit_camera(12.0)
    with V.Vdi(b, store="bf16") as hb:
        want_b = hb.render(cam, 96, 80)
        torch.cuda.synchronize()
    with V.Vdi(sources[0], store="bf16") as h:
        want_a = h.render(cam, 96, 80, d_i=2.0, d_r=2.0)
        torch.cuda.synchronize()
        o1 = torch.empty((80, 96, 4), dtype=torch.float32, device="cuda")
        o2 = torch.empty((80, 96, 4), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        with serve.Server(2 ** 34, max_inflight=16, persistent=True) as srv:
            t = srv.submit(h, cam, 96, 80, 2.0, 2.0, o1)
            srv.drain()
            assert srv.poll(t) and srv.stats()["batches"] == 1
            h.replace_begin(b)
            t0 = time.time()
            while not h.replace_poll():
                assert time.time() - t0 < 20.0, "replacement did not complete"
                time.sleep(0.001)
            t = srv.submit(h, cam, 96, 80, 1.0, 0.0, o2)
            srv.drain()
            assert srv.poll(t) and srv.stats()["batches"] == 2
    assert torch.equal(o1, want_a) and torch.equal(o2, want_b)
    ne = oracle_check(b, oracle.dequant_bf16(b.rgba), cam, 96, 80, 1.0, 0.0, o2.cpu().numpy(), seed=2)
    assert ne >= 100, ne


def test_1080p_requests_through_both_engines():
    """Requests at the served workload's full size (1920 x 1080 frames of the
    1080p VDI, N_S = 50, FP16 colour): exact and D_I = 2 / D_R = 2, through
    the batched server and the persistent one, each equal to its vdi_render
    and matching the oracle on the stored colours."""
    from paper_2206_08660_amd import serve
    from paper_2206_08660_amd import vdi as V
    src = inputs.load_workload("1080p", keep_dvr=False)
    reqs = [(20.0, 1.0, 0.0), (-25.0, 2.0, 2.0)]
    with V.Vdi(src, store="f16") as h:
        want = [h.render(inputs.orbit_camera(y), 1920, 1080, di, dr) for (y, di, dr) in reqs]
        torch.cuda.synchronize()
        for persistent in (False, True):
            outs = [torch.empty((1080, 1920, 4), dtype=torch.float32, device="cuda") for _ in reqs]
            torch.cuda.synchronize()
            with serve.Server(2 ** 34, max_inflight=8, persistent=persistent) as srv:
                ts = [srv.submit(h, inputs.orbit_camera(y), 1920, 1080, di, dr, o) for (y, di, dr), o in zip(reqs, outs)]
                srv.drain()
                assert all(t is not None and srv.poll(t) for t in ts)
            for w, o in zip(want, outs):
                assert torch.equal(w, o), persistent
            say(f"[gpu] 1080p requests through the {'persistent' if persistent else 'batched'} server: equal to vdi_render")
    rgba = oracle.dequant_f16(src.rgba)
    for i, (y, di, dr) in enumerate(reqs):
        ne = oracle_check(src, rgba, inputs.orbit_camera(y), 1920, 1080, di, dr, outs[i].cpu().numpy(), n=1200, seed=i)
        say(f"[gpu] 1080p served request yaw {y}, D_I={di}, D_R={dr} vs oracle: {ne} non-empty pixels")
        assert ne >= 300, ne
