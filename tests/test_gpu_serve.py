"""Served form through the C ABI (needs an MI355X): each request's image is
the same alone (vdi_render) and in the mix of concurrently admitted
requests; admission by budget and slots; completion of every request."""
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


@pytest.fixture(scope="module")
def handles():
    from paper_2206_08660_amd import vdi as V
    srcs = [inputs.load_workload("tiny"), inputs.load_workload("720p", keep_dvr=False)]
    hs = [V.Vdi(srcs[0]), V.Vdi(srcs[1], store="f16")]
    yield hs
    for h in hs:
        h.close()


def test_mixed_requests_match_single_renders(handles):
    from paper_2206_08660_amd import serve
    rng = np.random.default_rng(3)
    reqs = []
    for i in range(48):
        hi = i % 2
        W, H = [(128, 128), (96, 64), (1280, 720), (640, 360)][(i // 2) % 4] if hi else [(128, 128), (70, 44)][i % 2]
        di, dr = [(1.0, 0.0), (2.0, 2.0), (1.0, 0.5), (4.0, 2.0)][i % 4]
        reqs.append((hi, float(rng.uniform(-30, 30)), W, H, di, dr))
    outs = [torch.full((H, W, 4), -1.0, dtype=torch.float32, device="cuda") for (_, _, W, H, _, _) in reqs]
    # The server writes with its own kernel: buffers must be ready before submission.
    torch.cuda.synchronize()
    with serve.Server(8 * 2 ** 30, max_inflight=64) as srv:
        tickets = []
        for (hi, yaw, W, H, di, dr), buf in zip(reqs, outs):
            t = srv.submit(handles[hi], inputs.orbit_camera(yaw), W, H, di, dr, buf)
            assert t is not None
            tickets.append(t)
        srv.drain()
        assert all(srv.poll(t) for t in tickets)
        st = srv.stats()
        say(f"[gpu] served {st['completed']} requests in {st['batches']} batches (largest {st['peak_batch']}), "
            f"peak in flight {st['peak_inflight']}")
        assert st["completed"] == len(reqs) and st["inflight"] == 0 and st["queued"] == 0
        assert st["peak_inflight"] > 1 and 1 <= st["batches"] <= len(reqs) and st["peak_batch"] >= 1
    for (hi, yaw, W, H, di, dr), buf in zip(reqs, outs):
        alone = handles[hi].render(inputs.orbit_camera(yaw), W, H, di, dr)
        torch.cuda.synchronize()
        a, b = alone.cpu().numpy(), buf.cpu().numpy()
        assert np.array_equal(a, b), (hi, yaw, W, H, di, dr, np.abs(a - b).max())


def test_admission_by_budget_and_slots(handles):
    from paper_2206_08660_amd import serve
    one = 1280 * 720 * 16
    with serve.Server(2 * one + 100, max_inflight=8) as srv:
        bufs = [torch.empty((720, 1280, 4), dtype=torch.float32, device="cuda") for _ in range(3)]
        cam = inputs.orbit_camera(10.0)
        t1 = srv.submit(handles[1], cam, 1280, 720, 1.0, 0.0, bufs[0])
        t2 = srv.submit(handles[1], cam, 1280, 720, 1.0, 0.0, bufs[1])
        assert t1 is not None and t2 is not None
        # A third one does not fit the budget until the first two are done.
        t3 = srv.submit(handles[1], cam, 1280, 720, 1.0, 0.0, bufs[2])
        if t3 is None:
            assert srv.stats()["rejected_budget"] >= 1
            srv.drain()
            t3 = srv.submit(handles[1], cam, 1280, 720, 1.0, 0.0, bufs[2])
        assert t3 is not None
        srv.drain()
    with serve.Server(2 ** 34, max_inflight=1) as srv:
        b = [torch.empty((128, 128, 4), dtype=torch.float32, device="cuda") for _ in range(2)]
        t = srv.submit(handles[0], inputs.orbit_camera(5.0), 128, 128, 1.0, 0.0, b[0])
        t2 = srv.submit(handles[0], inputs.orbit_camera(5.0), 128, 128, 1.0, 0.0, b[1])
        if t2 is None:
            assert srv.stats()["rejected_slots"] >= 1
        srv.drain()
        assert srv.poll(t)
        assert srv.stats()["completed"] >= 1
        srv.reset_stats()
        st = srv.stats()
        assert st["completed"] == 0 and st["submitted"] == 0 and st["batches"] == 0
        assert st["peak_inflight"] == 0 and st["inflight"] == 0


def test_open_loop_trace_small(handles):
    """A short Poisson trace: every request completes and matches its single render."""
    from paper_2206_08660_amd import serve
    arrivals, which, yaw, outsel = serve.make_trace(60, 2000.0, seed=11, nvdi=2)
    bases = [0.0, 0.0]
    keep = (0, 17, 42, 59)
    lat, makespan, stats, outs = serve.run_served(handles, bases, (arrivals, which, yaw, outsel), 2 ** 34, 32, keep=keep)
    assert sorted(outs) == list(keep) and (lat >= 0).all() and stats["completed"] == 60
    for i in keep:
        W, H, di, dr = serve.OUTPUTS[int(outsel[i])]
        alone = handles[int(which[i])].render(inputs.orbit_camera(float(yaw[i]), bases[int(which[i])]), W, H, di, dr)
        torch.cuda.synchronize()
        assert np.array_equal(alone.cpu().numpy(), outs[i].cpu().numpy())
