"""Drivers of the served-form and paced-session measurements, shared by
bench.py and the GPU tests (not part of the library).

Served workload: four resident VDIs (two 1280x720 / N_S=20 and two
1920x1080 / N_S=50, generating views 90 degrees apart, FP16 colour), 2000
requests with viewpoint deviation U[0, 30] degrees with random sign, output
uniform over {1280x720 exact, 1920x1080 exact, 1920x1080 D_I=2/D_R=2},
admission budget 64 GiB.  Arrivals are Poisson at 600 requests/s (latency)
and then all at t = 0 (throughput at saturation).  Each trace is also
rendered one request at a time with vdi_render for comparison.  Arrival
times are drawn in advance (open loop); a request's latency runs from its
arrival to the moment the host sees it complete.

Paced session: a camera path rendered with D_I chosen by the PI controller
(vdi_pace_*), fed the GPU time of each frame (HIP events on the render
stream).
"""
from __future__ import annotations

import contextlib
import gc
import time
from typing import Callable, Optional, Sequence

import numpy as np

from paper_2206_08660_amd import vdi as V
from paper_2206_08660_amd.pace import Pace
from paper_2206_08660_amd.serve import Server

TRACE_SEED = 2005
OUTPUTS = [(1280, 720, 1.0, 0.0), (1920, 1080, 1.0, 0.0), (1920, 1080, 2.0, 2.0)]


def make_trace(n: int = 2000, rate: float = 600.0, seed: int = TRACE_SEED, nvdi: int = 4):
    """Pre-drawn request trace: arrival times, VDI index, yaw, output choice."""
    rng = np.random.Generator(np.random.PCG64(seed))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n))
    which = rng.integers(0, nvdi, size=n)
    yaw = rng.uniform(0.0, 30.0, size=n) * rng.choice([-1.0, 1.0], size=n)
    out = rng.integers(0, len(OUTPUTS), size=n)
    return arrivals, which, yaw, out


@contextlib.contextmanager
def _no_gc():
    """Timed loops run without Python's cyclic garbage collector, whose
    occasional full passes would stall the host loop for tens of ms."""
    was = gc.isenabled()
    gc.collect()
    gc.disable()
    try:
        yield
    finally:
        if was:
            gc.enable()


def _percentiles(lat):
    lat = np.asarray(lat) * 1e3
    return {"p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_ms": round(float(lat.mean()), 3), "max_ms": round(float(lat.max()), 3)}


def load_vdis(store: str = "f16", log: Callable = print):
    import inputs
    srcs = []
    for name in ("720p", "1080p"):
        for base in (0.0, 90.0):
            srcs.append((name, base, inputs.load_workload(name, base_deg=base, verbose=True, keep_dvr=False)))
            log(f"loaded {name} base {base:g}")
    return srcs


def run_served(handles, bases, trace, budget: int, max_inflight: int, keep=(), server: Optional[Server] = None,
               log: Callable = print):
    """Open-loop served run; returns (latencies [s], makespan [s], stats, {request: image} for `keep`).

    Output images come from buffers allocated before the clock starts and
    reused once their request is done; the images of the requests in `keep`
    are retained instead.  With `server` the run uses that (already warm)
    server, whose counters are reset first; otherwise a new one."""
    import torch

    import inputs
    arrivals, which, yaw, outsel = trace
    n = len(arrivals)
    keep = set(int(i) for i in keep)
    counts = np.bincount(np.asarray(outsel, dtype=np.int64), minlength=len(OUTPUTS))
    pool = {k: [torch.empty((OUTPUTS[k][1], OUTPUTS[k][0], 4), dtype=torch.float32, device="cuda")
                for _ in range(min(max_inflight, int(counts[k])) + len(keep))] for k in range(len(OUTPUTS))}
    cams = [inputs.orbit_camera(float(yaw[i]), bases[int(which[i])]) for i in range(n)]
    torch.cuda.synchronize()
    lat = np.zeros(n)
    out_of = {}
    own = server is None
    srv = Server(budget, max_inflight) if own else server
    srv.reset_stats()
    try:
        with _no_gc():
            pending = {}
            nxt = 0
            done_count = 0
            t0 = time.perf_counter()
            while done_count < n:
                now = time.perf_counter() - t0
                # admit every request that has arrived, while it fits
                while nxt < n and arrivals[nxt] <= now:
                    k = int(outsel[nxt])
                    if not pool[k]:
                        break
                    W, H, di, dr = OUTPUTS[k]
                    buf = pool[k].pop()
                    t = srv.submit(handles[int(which[nxt])], cams[nxt], W, H, di, dr, buf)
                    if t is None:
                        pool[k].append(buf)
                        break
                    pending[t] = (nxt, k, buf)
                    nxt += 1
                for t in list(pending):
                    if srv.poll(t):
                        i, k, buf = pending.pop(t)
                        lat[i] = (time.perf_counter() - t0) - arrivals[i]
                        if i in keep:
                            out_of[i] = buf
                        else:
                            pool[k].append(buf)
                        done_count += 1
                if not pending and nxt < n:
                    wait = arrivals[nxt] - (time.perf_counter() - t0)
                    if wait > 2e-4:
                        time.sleep(wait - 1e-4)
            makespan = time.perf_counter() - t0
        stats = srv.stats()
    finally:
        if own:
            srv.close()
    return lat, makespan, stats, out_of


def run_unbatched(handles, bases, trace):
    """The same trace, one vdi_render at a time, synchronised per request."""
    import torch

    import inputs
    arrivals, which, yaw, outsel = trace
    n = len(arrivals)
    bufs = {k: torch.empty((OUTPUTS[k][1], OUTPUTS[k][0], 4), dtype=torch.float32, device="cuda")
            for k in range(len(OUTPUTS))}
    cams = [inputs.orbit_camera(float(yaw[i]), bases[int(which[i])]) for i in range(n)]
    torch.cuda.synchronize()
    lat = np.zeros(n)
    with _no_gc():
        t0 = time.perf_counter()
        for i in range(n):
            wait = arrivals[i] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            k = int(outsel[i])
            W, H, di, dr = OUTPUTS[k]
            handles[int(which[i])].render(cams[i], W, H, di, dr, out=bufs[k])
            torch.cuda.synchronize()
            lat[i] = (time.perf_counter() - t0) - arrivals[i]
        makespan = time.perf_counter() - t0
    return lat, makespan


def idle_overhead(srv, vdi: "V.Vdi", cam, size: int = 128, n: int = 200) -> dict:
    """Fixed cost of one small request on an idle GPU: a size x size exact
    frame submitted to the server (submission to the client seeing it done),
    the same frame through vdi_render plus a stream synchronisation, and the
    render kernel's own time (HIP events around vdi_render).  What the served
    latency adds over the kernel is the per-request cost that a kernel
    resident on the GPU, taking requests from a queue, could at most remove."""
    import torch
    out = torch.empty((size, size, 4), dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream()
    served, direct, kernel = [], [], []
    # The three are interleaved, one of each per round, so that clock and
    # power changes over the run affect them alike.
    with _no_gc():
        for _ in range(n):
            t0 = time.perf_counter()
            t = srv.submit(vdi, cam, size, size, 1.0, 0.0, out)
            assert t is not None, "small request rejected"
            while not srv.poll(t):
                time.sleep(0)
            served.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            vdi.render(cam, size, size, 1.0, 0.0, out=out, stream=s)
            s.synchronize()
            direct.append(time.perf_counter() - t0)
            # The second render is launched while the first one runs, so the
            # events around it time the kernel and not the host's preparation.
            e1, e2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            vdi.render(cam, size, size, 1.0, 0.0, out=out, stream=s)
            e1.record(s)
            vdi.render(cam, size, size, 1.0, 0.0, out=out, stream=s)
            e2.record(s)
            e2.synchronize()
            kernel.append(e1.elapsed_time(e2) * 1e-3)
    med = lambda a: round(float(np.median(a)) * 1e3, 4)
    return {"request": f"{size}x{size} exact, 1080p VDI, one at a time on an idle GPU, {n} rounds of the three",
            "served_p50_ms": med(served), "vdi_render_and_sync_p50_ms": med(direct), "kernel_p50_ms": med(kernel),
            "served_minus_kernel_ms": round(med(served) - med(kernel), 4)}


def serve_benchmark(n: int = 2000, rate: float = 600.0, budget: int = 64 * 2 ** 30, max_inflight: int = 256,
                    log: Callable = print) -> dict:
    """Open-loop latency at `rate` requests/s, then throughput at saturation
    (all n requests present at t = 0), served and one request at a time."""
    import torch

    import inputs
    srcs = load_vdis(log=log)
    handles = [V.Vdi(s, store="f16") for _, _, s in srcs]
    bases = [b for _, b, _ in srcs]
    trace = make_trace(n, rate)
    px = sum(OUTPUTS[int(k)][0] * OUTPUTS[int(k)][1] for k in trace[3])
    # One long-running server; both paths are warmed on the first 64 requests.
    srv = Server(budget, max_inflight)
    warm = tuple(a[:64] for a in trace)
    run_served(handles, bases, (warm[0] * 0.0, *warm[1:]), budget, max_inflight, server=srv)
    run_unbatched(handles, bases, (warm[0] * 0.0, *warm[1:]))
    torch.cuda.synchronize()
    out = {"workload": "4 resident FP16 VDIs (2x 1280x720/N_S=20, 2x 1920x1080/N_S=50; V_O 0 and 90 deg); "
                       f"{n} requests, yaw U[0,30] deg +-, outputs 720p exact / 1080p exact / 1080p D_I=2,D_R=2; "
                       f"admission budget {budget / 2 ** 30:g} GiB, {max_inflight} slots"}
    for name, tr in ((f"poisson_{rate:g}_per_s", trace), ("saturation", (trace[0] * 0.0, *trace[1:]))):
        lat, makespan, stats, _ = run_served(handles, bases, tr, budget, max_inflight, server=srv, log=log)
        log(f"{name} served: {n} requests in {makespan:.2f}s, p50 {np.percentile(lat, 50)*1e3:.2f} ms, "
            f"p99 {np.percentile(lat, 99)*1e3:.2f} ms, {stats['batches']} batches (peak {stats['peak_batch']}), "
            f"peak in flight {stats['peak_inflight']}")
        ulat, umake = run_unbatched(handles, bases, tr)
        log(f"{name} unbatched: {n} requests in {umake:.2f}s, p50 {np.percentile(ulat, 50)*1e3:.2f} ms, "
            f"p99 {np.percentile(ulat, 99)*1e3:.2f} ms")
        out[name] = {
            "served": {**_percentiles(lat), "Mpixels_per_s": round(px / makespan / 1e6, 1),
                       "requests_per_s": round(n / makespan, 1), "batches": stats["batches"],
                       "peak_batch": stats["peak_batch"], "peak_inflight": stats["peak_inflight"],
                       "peak_bytes_in_flight": stats["peak_bytes_in_flight"],
                       "rejected_budget": stats["rejected_budget"], "rejected_slots": stats["rejected_slots"]},
            "unbatched": {**_percentiles(ulat), "Mpixels_per_s": round(px / umake / 1e6, 1),
                          "requests_per_s": round(n / umake, 1)},
        }
    out["idle_small_request"] = idle_overhead(srv, handles[2], inputs.orbit_camera(20.0, bases[2]))
    log(f"idle small request: {out['idle_small_request']}")
    srv.close()
    out["persistent"] = persistent_benchmark(handles, bases, trace, budget, max_inflight, px, log=log)
    for h in handles:
        h.close()
    return out


def persistent_benchmark(handles, bases, trace, budget: int, max_inflight: int, px: int, log: Callable = print):
    """The same traces served by one persistent kernel (vdi_server_create_persistent),
    and the idle small request through it."""
    import torch

    import inputs
    n = len(trace[0])
    srv = Server(budget, max_inflight, persistent=True)
    warm = tuple(a[:64] for a in trace)
    run_served(handles, bases, (warm[0] * 0.0, *warm[1:]), budget, max_inflight, server=srv)
    torch.cuda.synchronize()
    out = {"engine": "one persistent kernel (vdi_server_create_persistent), 5 wavefronts per SIMD; the same traces"}
    for name, tr in ((f"poisson_{600:g}_per_s", trace), ("saturation", (trace[0] * 0.0, *trace[1:]))):
        lat, makespan, stats, _ = run_served(handles, bases, tr, budget, max_inflight, server=srv, log=log)
        log(f"{name} persistent: {n} requests in {makespan:.2f}s, p50 {np.percentile(lat, 50)*1e3:.2f} ms, "
            f"p99 {np.percentile(lat, 99)*1e3:.2f} ms, {stats['batches']} launches")
        out[name] = {**_percentiles(lat), "Mpixels_per_s": round(px / makespan / 1e6, 1),
                     "requests_per_s": round(n / makespan, 1), "launches": stats["batches"],
                     "peak_inflight": stats["peak_inflight"]}
    # One small request at a time on an otherwise idle GPU (the launch stays resident between them).
    cam = inputs.orbit_camera(20.0, bases[2])
    o = torch.empty((128, 128, 4), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    served = []
    with _no_gc():
        for _ in range(200):
            t0 = time.perf_counter()
            t = srv.submit(handles[2], cam, 128, 128, 1.0, 0.0, o)
            assert t is not None, "small request rejected"
            while not srv.poll(t):
                time.sleep(0)
            served.append(time.perf_counter() - t0)
    out["idle_small_request_p50_ms"] = round(float(np.median(served)) * 1e3, 4)
    log(f"idle small request, persistent: {out['idle_small_request_p50_ms']} ms")
    # Each output of the mix alone on an idle GPU (1080p VDI at 20 deg):
    # through the persistent launch, then (after it has ended) vdi_render + sync.
    single = {}
    for k, (W, H, di, dr) in enumerate(OUTPUTS):
        buf = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        ts = []
        with _no_gc():
            for _ in range(30):
                t0 = time.perf_counter()
                t = srv.submit(handles[2], cam, W, H, di, dr, buf)
                while not srv.poll(t):
                    time.sleep(0)
                ts.append(time.perf_counter() - t0)
        single[f"{W}x{H},D_I={di:g},D_R={dr:g}"] = {"persistent_ms": round(float(np.median(ts[5:])) * 1e3, 4)}
    srv.close()
    s = torch.cuda.current_stream()
    for k, (W, H, di, dr) in enumerate(OUTPUTS):
        buf = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
        ts = []
        with _no_gc():
            for _ in range(30):
                t0 = time.perf_counter()
                handles[2].render(cam, W, H, di, dr, out=buf, stream=s)
                s.synchronize()
                ts.append(time.perf_counter() - t0)
        single[f"{W}x{H},D_I={di:g},D_R={dr:g}"]["vdi_render_and_sync_ms"] = round(float(np.median(ts[5:])) * 1e3, 4)
    out["single_requests_idle"] = single
    log(f"single requests, persistent vs direct: {single}")
    return out


def profile_saturation(n: int = 2000, budget: int = 64 * 2 ** 30, max_inflight: int = 256, log: Callable = print):
    """The saturation trace, served only, after a warm-up of 64 requests (a
    short run to record under a kernel trace)."""
    import torch
    srcs = load_vdis(log=log)
    handles = [V.Vdi(s, store="f16") for _, _, s in srcs]
    bases = [b for _, b, _ in srcs]
    trace = make_trace(n)
    trace = (trace[0] * 0.0, *trace[1:])
    srv = Server(budget, max_inflight)
    run_served(handles, bases, tuple(a[:64] for a in trace), budget, max_inflight, server=srv)
    torch.cuda.synchronize()
    time.sleep(0.05)   # a gap that marks the start of the timed trace in a kernel trace
    lat, makespan, stats, _ = run_served(handles, bases, trace, budget, max_inflight, server=srv, log=log)
    log(f"saturation served: {n} requests in {makespan:.3f}s, {stats['batches']} batches")
    srv.close()
    for h in handles:
        h.close()


def run_session(vdi: "V.Vdi", cams: Sequence, width: int, height: int, d_r: float, pace: Pace, out=None,
                stream=None, keep=()):
    """Render cams in order with D_I from `pace`; returns [(D_I, frame_ms)]
    per frame, and with `keep` also {frame index: image} of those frames."""
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    if out is None:
        out = torch.empty((height, width, 4), dtype=torch.float32, device="cuda")
    log = []
    kept = {}
    for cam in cams:
        d_i = pace.d_i
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        vdi.render(cam, width, height, d_i, d_r, out=out, stream=s)
        e1.record(s)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        log.append((d_i, ms))
        if len(log) - 1 in keep:
            kept[len(log) - 1] = out.clone()
        pace.update(ms)
    return (log, kept) if keep else log


def run_served_session(srv, vdi: "V.Vdi", cams: Sequence, width: int, height: int, d_r: float, pace: Pace,
                       keep=()):
    """An interactive client of a server: each frame is submitted as a
    request of the paced session `pace` once the previous one is done, with
    the D_I the server takes from the session.  Returns [(D_I, latency ms)]
    per frame (latency from submission to the client seeing it done), and
    with `keep` also {frame index: image} of those frames."""
    import torch
    out = torch.empty((height, width, 4), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    log, kept = [], {}
    for cam in cams:
        t0 = time.perf_counter()
        r = srv.submit_paced(vdi, cam, width, height, pace, d_r, out)
        assert r is not None, "paced request rejected"
        ticket, d_i = r
        while not srv.poll(ticket):
            time.sleep(0)
        log.append((d_i, 1e3 * (time.perf_counter() - t0)))
        if len(log) - 1 in keep:
            kept[len(log) - 1] = out.clone()
    return (log, kept) if keep else log
