#!/usr/bin/env python3
"""Benchmark of VDI raycasting on one MI355X.

One step renders the 1920x1080 VDI with N_S = 50 (the turbulence-shell
workload) at the ten viewpoints 0, 5, ..., 45 degrees about the volume's y
axis, each in three modes: exact (D_I = 1, D_R = 0) and the preview modes
D_I = 2 / D_R = 2 and D_I = 4 / D_R = 2, all to a 1920x1080 output: 30 frames.
The VDI is resident in HBM before timing starts (its generation on the host
is never timed).  The frames of a step are independent: a step is two
vdi_render_batch calls (alternate frames) on two streams; per-frame times
come from a separate pass that renders them one at a time on one stream.

Printed: one JSON line with Mpixels/s over the step, the roofline of the
dominant kernel (algorithmic bytes per launch from the instrumented
counter kernel / launch time from HIP events on the launch stream), the FP16
and BF16 storage forms, the served form (continuous batching) and the FP64
CPU oracle timed on a bounded pixel sample of the same workload.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
W, H = 1920, 1080
ANGLES = [5.0 * i for i in range(10)]
MODES = [(1.0, 0.0), (2.0, 2.0), (4.0, 2.0)]
METRIC = "VDI render Mpixels/s + HBM GB/s fraction; p50/p99 frame latency (served)"
KERNEL_SRCS = [os.path.join(ROOT, "paper_2206_08660_amd", "csrc", f) for f in ("vdi_kernels.hip", "vdi_trace.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "render_exact_1080p_traffic.json")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--skip-cpu-baseline", action="store_true")
    p.add_argument("--skip-served", action="store_true")
    p.add_argument("--skip-precision", action="store_true")
    p.add_argument("--skip-replace", action="store_true")
    p.add_argument("--skip-paced", action="store_true")
    p.add_argument("--skip-generation", action="store_true")
    p.add_argument("--skip-quality", action="store_true")
    p.add_argument("--skip-search", action="store_true")
    p.add_argument("--profile-pass", action="store_true",
                   help="short run for rocprofv3: one 1 GiB copy (counter calibration) and one exact render per angle")
    p.add_argument("--profile-preview", action="store_true",
                   help="short run for rocprofv3: one D_I=2/D_R=2 and one D_I=4/D_R=2 render per angle")
    p.add_argument("--profile-generation", action="store_true",
                   help="short run for rocprofv3: one 1 GiB copy, then two GPU generations of the 720p VDI "
                        "(1280x720, N_S=20, generating view 0 deg), the second the one to read")
    p.add_argument("--profile-served", action="store_true",
                   help="short run for rocprofv3: the served saturation trace (2000 requests) after a warm-up")
    return p.parse_args()


def kernel_hash() -> str:
    """Hash of the render kernel's sources: stored counter figures apply only while it matches."""
    h = hashlib.sha1()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:12]


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU design is described, "
              "not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import inputs
    from paper_2206_08660_amd import vdi as V

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.profile_generation:
        profile_generation(torch, V)
        return
    if args.profile_served:
        from tests import harness
        harness.profile_saturation(log=log)
        return

    t = time.time()
    src = inputs.load_workload("1080p", verbose=True)
    log(f"workload ready in {time.time() - t:.1f}s: VDI {src.width}x{src.height}x{src.ns}, "
        f"{int(src.count.sum())} supersegments")
    torch.cuda.synchronize()
    t_up = time.perf_counter()
    h = V.Vdi(src)
    torch.cuda.synchronize()
    upload_s = time.perf_counter() - t_up
    info = h.info()
    log(f"resident: {info.device_bytes / 2**30:.2f} GiB, vdi_create (host -> HBM, brick scatter, grid) {upload_s * 1e3:.0f} ms")
    out = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
    cams = {th: inputs.orbit_camera(th) for th in ANGLES}
    renders = [(th, di, dr) for th in ANGLES for (di, dr) in MODES]

    if args.profile_pass:
        a = torch.empty(2 ** 28, dtype=torch.float32, device="cuda").fill_(1.0)   # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        for th in ANGLES:
            h.render(cams[th], W, H, 1.0, 0.0, out=out)
        torch.cuda.synchronize()
        log("profile pass done")
        return
    if args.profile_preview:
        for th in ANGLES:
            for di, dr in MODES:
                if dr > 0.0:
                    h.render(cams[th], W, H, di, dr, out=out)
        torch.cuda.synchronize()
        log("preview profile pass done")
        return

    # The 30 frames of a step are independent.  The timed steps render them
    # with vdi_render_batch, alternate frames on two streams (one output
    # buffer per frame): each call puts all its exact frames in one launch,
    # all its preview frames in another and their upsampling in a third, so
    # the long rays at the end of one frame run beside other frames' tiles,
    # and the two streams overlap the tails of the launches.  Every frame is
    # bit-identical to a vdi_render of it.
    streams = [stream, torch.cuda.Stream()]
    step_outs = [torch.empty_like(out) for _ in renders]

    def step(handle):
        start = torch.cuda.Event()
        start.record(stream)
        streams[1].wait_event(start)
        for half in (0, 1):
            V.render_batch([(handle, cams[th], W, H, di, dr, step_outs[k])
                            for k, (th, di, dr) in enumerate(renders) if k % 2 == half], stream=streams[half])
        joined = torch.cuda.Event()
        joined.record(streams[1])
        stream.wait_event(joined)

    for _ in range(args.warmup):
        step(h)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} steps done; timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(h)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = 1e3 * elapsed / args.steps
    mpix = len(renders) * W * H * args.steps / elapsed / 1e6
    log(f"step {ms_step:.3f} ms, {mpix:.1f} Mpixels/s (vdi_render_batch, 2 streams)")

    # Per-frame times: the same frames one at a time on one stream, each
    # bracketed by HIP events on that stream (the GPU to itself), averaged
    # over the repetitions.
    reps = max(3, min(args.steps, 10))
    evs = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in renders]
           for _ in range(reps)]
    # One untimed pass first: measured, the first frame-by-frame pass after
    # the batched steps runs its D_I = 2 frames about 30% slower than the
    # passes after it (exact frames are not affected).
    for (th, di, dr) in renders:
        h.render(cams[th], W, H, di, dr, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in range(reps):
        for k, (th, di, dr) in enumerate(renders):
            evs[i][k][0].record(stream)
            h.render(cams[th], W, H, di, dr, out=out)
            evs[i][k][1].record(stream)
    torch.cuda.synchronize()
    seq_ms_step = 1e3 * (time.perf_counter() - t1) / reps
    per = {r: float(np.mean([evs[i][k][0].elapsed_time(evs[i][k][1]) for i in range(reps)]))
           for k, r in enumerate(renders)}
    per_p99 = {r: float(np.percentile([evs[i][k][0].elapsed_time(evs[i][k][1]) for i in range(reps)], 99))
               for k, r in enumerate(renders)}
    log(f"one stream, frame by frame: {seq_ms_step:.3f} ms per step")

    # The same exact frames with the 256 MB Infinity Cache flushed before each
    # (a 512 MB buffer written between frames).
    flush = torch.empty(2 ** 27, dtype=torch.float32, device="cuda")
    flushed = {}
    for th in ANGLES:
        ts = []
        for _ in range(5):
            flush.fill_(float(th))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            h.render(cams[th], W, H, 1.0, 0.0, out=out)
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        flushed[th] = float(np.median(ts))
    del flush
    # A measured bandwidth peak: a 1 GiB device-to-device copy (2 GiB moved).
    a = torch.empty(2 ** 28, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    cts = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.copy_(a)
        e1.record(stream)
        torch.cuda.synchronize()
        cts.append(e0.elapsed_time(e1))
    copy_gbs = 2 * a.numel() * 4 / (float(np.median(cts)) / 1e3) / 1e9
    del a, b
    log(f"copy kernel: {copy_gbs:.0f} GB/s")
    exact_ms = {th: per[(th, 1.0, 0.0)] for th in ANGLES}
    mode_ms = {f"D_I={di:g},D_R={dr:g}": sum(per[(th, di, dr)] for th in ANGLES) for (di, dr) in MODES}
    log("per-mode ms (sum over 10 angles): " + ", ".join(f"{k}: {v:.3f}" for k, v in mode_ms.items()))

    # Algorithmic bytes of each exact frame (instrumented kernel, same options
    # as the timed one): per list a ray entered, its count byte and all its
    # (f, b) pairs; per supersegment composited, its colour; plus the output.
    count_d = torch.from_numpy(np.ascontiguousarray(src.count)).cuda().to(torch.int64)
    balg = {}
    visits = {}
    for th in ANGLES:
        _, tl, ts, st = h.render_counters(cams[th], W, H, ess=True)
        touched = tl.bool()
        balg[th] = int(touched.sum().item() + 8 * count_d[touched].sum().item() + 16 * ts.sum(dtype=torch.int64).item()
                       + 16 * W * H)
        sums = st.reshape(-1, 2).to(torch.int64).sum(dim=0).tolist()
        visits[th] = (int(sums[0]), int(sums[1]))
        del tl, ts, st
    torch.cuda.synchronize()
    total_b = sum(balg.values())
    total_s = sum(exact_ms.values()) / 1e3
    total_flushed_s = sum(flushed.values()) / 1e3
    # The roofline fraction takes the MALL-flushed frame times (nothing of the
    # VDI left in the 256 MB Infinity Cache); the warm figure sits beside it.
    achieved = total_b / total_flushed_s / 1e9
    achieved_warm = total_b / total_s / 1e9
    exact_mpix = len(ANGLES) * W * H / total_s / 1e6
    log(f"exact frames: {exact_mpix:.1f} Mpixels/s; roofline {achieved:.0f} GB/s flushed, {achieved_warm:.0f} GB/s warm")
    # Preview frames: algorithmic bytes from the instrumented preview kernel
    # (per list sampled its count byte and (f, b) pairs, per supersegment
    # composited its colour, 4 bytes per grid cell read, the low-res image
    # written and read back by the upsampling, the output written) against
    # the whole render (preview kernel + upsampling), warm.
    preview_roof = {}
    preview_bytes_total = {}
    for (di, dr) in MODES:
        if dr == 0.0:
            continue
        pb, pms, samples = 0, 0.0, 0
        for th in ANGLES:
            lo_img, tl, ts, tc, st = h.preview_counters(cams[th], W, H, di, dr)
            touched = tl.bool()
            lw, lh = lo_img.shape[1], lo_img.shape[0]
            pb += int(touched.sum().item() + 8 * count_d[touched].sum().item()
                      + 16 * ts.sum(dtype=torch.int64).item() + 4 * tc.sum(dtype=torch.int64).item()
                      + 16 * (2 * lw * lh + W * H))
            samples += int(st[..., 0].sum(dtype=torch.int64).item())
            pms += per[(th, di, dr)]
            del lo_img, tl, ts, tc, st
        preview_bytes_total[(di, dr)] = pb
        preview_roof[f"D_I={di:g},D_R={dr:g}"] = {
            "algorithmic_MB_per_frame": round(pb / len(ANGLES) / 1e6, 2), "ms_per_frame": round(pms / len(ANGLES), 4),
            "achieved_GBs": round(pb / (pms / 1e3) / 1e9, 1), "frac": round(pb / (pms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "samples_M_per_frame": round(samples / len(ANGLES) / 1e6, 3)}
    torch.cuda.synchronize()
    log("preview roofline: " + ", ".join(f"{k} {v['achieved_GBs']} GB/s ({v['frac']})" for k, v in preview_roof.items()))
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("kernel_src_sha1") == kernel_hash():
            traffic = tr.get("bytes_per_launch")
    breakdown = {
        "exact_ms": {f"{th:g}": round(exact_ms[th], 4) for th in ANGLES},
        "exact_balg_MB": {f"{th:g}": round(balg[th] / 1e6, 2) for th in ANGLES},
        "exact_GBs": {f"{th:g}": round(balg[th] / exact_ms[th] / 1e6, 1) for th in ANGLES},
        "exact_hbm_frac": {f"{th:g}": round(balg[th] / exact_ms[th] / 1e6 / HBM_PEAK_GBS, 4) for th in ANGLES},
        "exact_ms_p99": {f"{th:g}": round(per_p99[(th, 1.0, 0.0)], 4) for th in ANGLES},
        "exact_ms_mall_flushed": {f"{th:g}": round(flushed[th], 4) for th in ANGLES},
        "exact_hbm_frac_mall_flushed": {f"{th:g}": round(balg[th] / flushed[th] / 1e6 / HBM_PEAK_GBS, 4)
                                        for th in ANGLES},
        "exact_list_visits_M": {f"{th:g}": round(visits[th][0] / 1e6, 2) for th in ANGLES},
        "exact_pieces_M": {f"{th:g}": round(visits[th][1] / 1e6, 2) for th in ANGLES},
        "preview_D_I2_D_R2_ms": {f"{th:g}": round(per[(th, 2.0, 2.0)], 4) for th in ANGLES},
        "preview_D_I4_D_R2_ms": {f"{th:g}": round(per[(th, 4.0, 2.0)], 4) for th in ANGLES},
        "mode_ms_per_10_angles": {k: round(v, 3) for k, v in mode_ms.items()},
        "fps_exact": {f"{th:g}": round(1e3 / exact_ms[th], 1) for th in ANGLES},
    }
    result = {
        "metric": METRIC,
        "value": round(mpix, 2),
        "unit": "Mpixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded 1024x1024x512 f32 turbulence-shell volume -> VDI by Eq. 1 + Alg. S1)",
        "config": {"workload": "1080p VDI 1920x1080, N_S=50, FP32 colour; 10 viewpoints 0-45 deg x "
                               "{exact, D_I=2/D_R=2, D_I=4/D_R=2}; output 1920x1080",
                   "frames_per_step": len(renders), "step_calls": "vdi_render_batch x 2 (alternate frames), 2 streams", "vdi_supersegments": int(info.supersegments),
                   "vdi_device_GiB": round(info.device_bytes / 2 ** 30, 3),
                   "preview_rays": {f"D_I={di:g}": int(np.prod(V.lowres_size(W, H, di))) for (di, dr) in MODES if dr > 0},
                   "vdi_create_ms": round(upload_s * 1e3, 1)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "k_render_exact (exact mode, FP32 colour, ESS, window search)",
                     "timing": "MALL-flushed launches (512 MB written before each), one at a time on one stream, "
                               "mean over the 10 viewpoints; warm: the frame-by-frame pass",
                     "algorithmic_bytes_per_launch": int(total_b / len(ANGLES)),
                     "launch_ms": round(1e3 * total_flushed_s / len(ANGLES), 4),
                     "achieved_warm": round(achieved_warm, 1), "frac_warm": round(achieved_warm / HBM_PEAK_GBS, 4),
                     "launch_ms_warm": round(1e3 * total_s / len(ANGLES), 4),
                     "copy_kernel_GBs": round(copy_gbs, 1),
                     "frac_of_copy_kernel": round(achieved / copy_gbs, 4)},
        "preview_roofline": preview_roof,
        # The whole timed step: the algorithmic bytes of its 30 frames (exact
        # and preview, as above) over the step time, the two streams together.
        "step_roofline": {"algorithmic_MB_per_step": round((total_b + sum(preview_bytes_total.values())) / 1e6, 1),
                          "achieved_GBs": round((total_b + sum(preview_bytes_total.values())) / (ms_step / 1e3) / 1e9, 1),
                          "frac": round((total_b + sum(preview_bytes_total.values())) / (ms_step / 1e3) / 1e9
                                        / HBM_PEAK_GBS, 4)},
        "exact_only": {"Mpixels_per_s": round(exact_mpix, 1), "frames_per_s": round(len(ANGLES) / total_s, 1)},
        "one_stream": {"ms_per_step": round(seq_ms_step, 4),
                       "Mpixels_per_s": round(len(renders) * W * H / seq_ms_step / 1e3, 1),
                       "sum_of_frame_ms": round(sum(per.values()), 4), "repetitions": reps},
        "breakdown": breakdown,
    }

    if not args.skip_search:
        result["search"] = search_leg(h, cams, out, stream, torch)
    if not args.skip_precision:
        result["precision"] = precision_leg(src, cams, out, exact_ms, torch, V)
    if not args.skip_served:
        result["served"] = served_leg(torch, V)
    if not args.skip_paced:
        result["paced"] = paced_leg(h, out, stream, np)
    # The quality leg renders the resident VDI of the step; the replacement leg swaps another one in.
    if not args.skip_quality:
        result["quality"] = quality_leg(src, h, cams, out, stream, torch, V)
    if not args.skip_replace:
        result["replacement"] = replace_leg(h, cams[20.0], out, stream, torch, V)
    if not args.skip_generation:
        result["generation"] = generation_leg(src, torch, V)
    h.close()
    if not args.skip_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline_leg(src, cams, per, result.get("precision"), np, torch, V)
    print(json.dumps(result), flush=True)


def search_leg(h, cams, out, stream, torch):
    """First-supersegment search strategies (Section 4.2, supplement Alg. S2 /
    Fig. 4): exact frames at the 10 viewpoints with each search, with and
    without empty-space skipping (the image is the same for all)."""
    res = {}
    for ess in (True, False):
        for search in ("window", "seeded", "binary", "linear"):
            ms = {f"{th:g}": round(_event_ms(lambda: h.render(cams[th], W, H, out=out, ess=ess, search=search),
                                             stream, torch, reps=3, warm=1), 4) for th in ANGLES}
            res[f"{search}{'' if ess else '_no_ess'}"] = {"sum_ms": round(sum(ms.values()), 3), "per_angle_ms": ms}
    w = res["window"]["sum_ms"]
    log("search (exact sweep, ms): " + ", ".join(f"{k} {v['sum_ms']}" for k, v in res.items()))
    res["speedup_window_vs_best_of_binary_linear"] = round(min(res["binary"]["sum_ms"], res["linear"]["sum_ms"]) / w, 2)
    res["speedup_seeded_vs_best_of_binary_linear"] = round(
        min(res["binary"]["sum_ms"], res["linear"]["sum_ms"]) / res["seeded"]["sum_ms"], 2)
    return res


def precision_leg(src, cams, out, exact_ms, torch, V):
    """FP16 / BF16 colour storage: exact-mode frame times against FP32."""
    import numpy as np
    res = {}
    stream = torch.cuda.current_stream()
    for fmt in ("f16", "bf16"):
        with V.Vdi(src, store=fmt) as hq:
            ms = {}
            for th in ANGLES:
                for _ in range(2):
                    hq.render(cams[th], W, H, out=out)
                ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(10)]
                for e0, e1 in ev:
                    e0.record(stream)
                    hq.render(cams[th], W, H, out=out)
                    e1.record(stream)
                torch.cuda.synchronize()
                ms[th] = float(np.mean([e0.elapsed_time(e1) for e0, e1 in ev]))
            res[fmt] = {"exact_ms_sum_10_angles": round(sum(ms.values()), 4),
                        "speedup_vs_f32": round(sum(exact_ms.values()) / sum(ms.values()), 3),
                        "device_GiB": round(hq.info().device_bytes / 2 ** 30, 3)}
        log(f"{fmt}: exact sweep {res[fmt]['exact_ms_sum_10_angles']:.3f} ms "
            f"(x{res[fmt]['speedup_vs_f32']} vs f32)")
    return res


def paced_leg(h, out, stream, np):
    """Frame-time-paced preview (PI controller on D_I, D_R = 2 fixed): the
    plant (frame time against D_I at three viewpoints), then a session of 80
    frames at 5 deg, 120 at 40 deg and 80 at 5 deg with the target set to 85%
    of the 40-degree frame at full resolution."""
    import inputs
    from paper_2206_08660_amd.pace import Pace
    from tests.harness import run_session
    d_r = 2.0
    fixed = lambda d: Pace(1e6, d_i_min=d, d_i_max=d, d_i_start=d)
    plant = {}
    for th in (5.0, 25.0, 40.0):
        cam = inputs.orbit_camera(th)
        plant[f"{th:g}"] = {f"{d:g}": round(float(np.median([t for _, t in run_session(
            h, [cam] * 10, W, H, d_r, fixed(d), out=out, stream=stream)][3:])), 4) for d in (1.0, 2.0, 4.0, 8.0)}
    target = 0.85 * plant["40"]["1"]
    easy, hard = inputs.orbit_camera(5.0), inputs.orbit_camera(40.0)
    with Pace(target, d_i_max=8.0) as p:
        trace = run_session(h, [easy] * 80 + [hard] * 120 + [easy] * 80, W, H, d_r, p, out=out, stream=stream)
    d_i = np.array([d for d, _ in trace])
    ms = np.array([t for _, t in trace])
    rel = np.abs(ms[100:200] / target - 1.0)
    res = {"workload": "1080p FP32 VDI, 1920x1080 preview with D_R = 2, D_I by the PI controller (kp 0.1, ki 0.3, "
                       "D_I in [1, 8]); 80 frames at 5 deg, 120 at 40 deg, 80 at 5 deg",
           "plant_frame_ms_by_deg_and_D_I": plant, "target_ms": round(target, 4),
           "easy_D_I_mean": round(float(d_i[10:80].mean()), 3), "easy_frame_ms_median": round(float(np.median(ms[10:80])), 4),
           "hard_D_I_mean": round(float(d_i[100:200].mean()), 3),
           "hard_frame_ms_median": round(float(np.median(ms[100:200])), 4),
           "hard_rel_err_median": round(float(np.median(rel)), 4), "hard_within_10pct": round(float(np.mean(rel < 0.1)), 3),
           "easy_again_D_I_mean": round(float(d_i[220:].mean()), 3)}
    log(f"paced: target {res['target_ms']} ms; hard view D_I {res['hard_D_I_mean']} at {res['hard_frame_ms_median']} ms, "
        f"easy view D_I {res['easy_D_I_mean']}; plant at 40 deg {plant['40']}")
    return res


def replace_leg(h, cam, out, stream, torch, V):
    """Double-buffered replacement: a second 1080p FP32 VDI (generated 90
    degrees away) is uploaded into the resident one from another thread while
    the main thread keeps rendering exact 1920x1080 frames."""
    import threading

    import numpy as np

    import inputs
    b = inputs.load_workload("1080p", base_deg=90.0, keep_dvr=False)

    def frame_ms(n):
        ts = []
        for _ in range(n):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            h.render(cam, W, H, out=out)
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return ts

    idle = frame_ms(20)
    call = {}

    def replace():
        t = time.perf_counter()
        h.replace_begin(b, stream=stream)
        call["ms"] = 1e3 * (time.perf_counter() - t)

    torch.cuda.synchronize()
    th = threading.Thread(target=replace)
    t0 = time.perf_counter()
    th.start()
    during = []
    while True:
        during += frame_ms(1)
        if not th.is_alive() and h.replace_poll():
            break
    swap_ms = 1e3 * (time.perf_counter() - t0)
    th.join()
    after = frame_ms(20)
    res = {"workload": "1080p FP32 VDI (2.3 GiB) replaced by one generated 90 deg away, from a second thread, "
                       "while rendering 1920x1080 exact frames at 20 deg",
           "begin_to_swap_ms": round(swap_ms, 1), "replace_begin_host_ms": round(call.get("ms", -1.0), 1),
           "frames_during_upload": len(during), "frame_ms_idle": round(float(np.median(idle)), 4),
           "frame_ms_during_upload": round(float(np.median(during)), 4),
           "frame_ms_after_swap": round(float(np.median(after)), 4)}
    log(f"replacement: swapped after {swap_ms:.0f} ms; {len(during)} frames meanwhile at "
        f"{res['frame_ms_during_upload']} ms (idle {res['frame_ms_idle']} ms)")
    return res


def _event_ms(fn, stream, torch, reps=5, warm=2):
    """Mean GPU time of fn() over reps launches, HIP events on the launch stream."""
    import numpy as np
    for _ in range(warm):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    return float(np.mean([e0.elapsed_time(e1) for e0, e1 in ev]))


def quality_leg(src, h, cams, out, stream, torch, V):
    """VDI renderings against DVR of the volume from the same viewpoint
    (Section 6, Figs. 7-9): SSIM / PSNR against the FP64 DVR at every
    viewpoint of the step (exact mode), the D_I x D_R grid at 30 degrees with
    frame times (the fps / quality trade-off), and frame times of DVR (FP64
    reference and FP32 shading) against exact VDI rendering with and without
    empty-space skipping, for the 1080p and the 720p workloads."""
    import numpy as np

    import inputs
    res = {}
    spec = inputs.WORKLOADS["1080p"]
    vol = inputs.make_volume(spec)
    dvol = torch.from_numpy(vol).cuda()
    del vol
    tf = "knots4"
    ref = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
    dvr_out = torch.empty_like(ref)
    per_angle = {}
    for th in ANGLES:
        V.dvr(dvol, src.bmin, src.bmax, cams[th], W, H, tf=tf, precision="f64", out=ref)
        h.render(cams[th], W, H, out=out)
        s, p = V.image_quality(out, ref)
        ms64 = _event_ms(lambda: V.dvr(dvol, src.bmin, src.bmax, cams[th], W, H, tf=tf, precision="f64",
                                       out=dvr_out), stream, torch, reps=2, warm=0)
        ms32 = _event_ms(lambda: V.dvr(dvol, src.bmin, src.bmax, cams[th], W, H, tf=tf, precision="f32",
                                       out=dvr_out), stream, torch)
        s32, p32 = V.image_quality(dvr_out, ref)
        vdi_ms = _event_ms(lambda: h.render(cams[th], W, H, out=out), stream, torch)
        vdi_noess = _event_ms(lambda: h.render(cams[th], W, H, out=out, ess=False), stream, torch)
        per_angle[f"{th:g}"] = {"ssim": round(s, 5), "psnr_db": round(p, 2), "vdi_ms": round(vdi_ms, 4),
                                "vdi_no_ess_ms": round(vdi_noess, 4), "dvr_f32_ms": round(ms32, 3),
                                "dvr_f64_ms": round(ms64, 2), "dvr_f32_psnr_vs_f64_db": round(p32, 1),
                                "speedup_vs_dvr_f32": round(ms32 / vdi_ms, 1)}
    res["1080p_exact_vs_dvr"] = per_angle
    log("quality 1080p exact: " + ", ".join(f"{k} deg SSIM {v['ssim']} PSNR {v['psnr_db']}" for k, v in per_angle.items()))
    th = 30.0
    V.dvr(dvol, src.bmin, src.bmax, cams[th], W, H, tf=tf, precision="f64", out=ref)
    grid = {}
    for di in (1.0, 2.0, 4.0):
        for dr in (0.0, 0.5, 1.0, 2.0, 4.0):
            h.render(cams[th], W, H, di, dr, out=out)
            s, p = V.image_quality(out, ref)
            ms = _event_ms(lambda: h.render(cams[th], W, H, di, dr, out=out), stream, torch)
            grid[f"D_I={di:g},D_R={dr:g}"] = {"ssim": round(s, 5), "psnr_db": round(p, 2), "ms": round(ms, 4),
                                              "fps": round(1e3 / ms, 1)}
    res["1080p_30deg_DI_x_DR"] = grid
    del dvol
    torch.cuda.empty_cache()
    # 720p workload: frame rates of exact VDI rendering (ESS on / off) against DVR.
    spec = inputs.WORKLOADS["720p"]
    s720 = inputs.load_workload("720p", keep_dvr=False)
    vol = inputs.make_volume(spec)
    dvol = torch.from_numpy(vol.view(np.int16)).cuda()
    del vol
    w7, h7 = spec["width"], spec["height"]
    o7 = torch.empty((h7, w7, 4), dtype=torch.float32, device="cuda")
    r7 = torch.empty_like(o7)
    row = {}
    with V.Vdi(s720) as h720:
        for th7 in (5.0, 15.0, 30.0, 45.0):
            cam = inputs.orbit_camera(th7)
            V.dvr(dvol, s720.bmin, s720.bmax, cam, w7, h7, tf=tf, precision="f64", out=r7)
            h720.render(cam, w7, h7, out=o7)
            s, p = V.image_quality(o7, r7)
            vdi_ms = _event_ms(lambda: h720.render(cam, w7, h7, out=o7), stream, torch)
            noess = _event_ms(lambda: h720.render(cam, w7, h7, out=o7, ess=False), stream, torch)
            d32 = _event_ms(lambda: V.dvr(dvol, s720.bmin, s720.bmax, cam, w7, h7, tf=tf, precision="f32", out=r7),
                            stream, torch)
            row[f"{th7:g}"] = {"ssim": round(s, 5), "psnr_db": round(p, 2), "vdi_ms": round(vdi_ms, 4),
                               "vdi_no_ess_ms": round(noess, 4), "dvr_f32_ms": round(d32, 3),
                               "speedup_vs_dvr_f32": round(d32 / vdi_ms, 1)}
    res["720p_exact_vs_dvr"] = row
    # GPU against the CPU FP64 references (all host threads) on one 1280x720 frame at 30 deg:
    # DVR (the generator's own DVR pass on the CPU) and SSIM / PSNR (numpy on the CPU).
    from oracle import quality as Q
    cam = inputs.orbit_camera(30.0)
    gpu_dvr = _event_ms(lambda: V.dvr(dvol, s720.bmin, s720.bmax, cam, w7, h7, tf=tf, precision="f64", out=r7),
                        stream, torch, reps=3, warm=1)
    with V.Vdi(s720) as h720:
        h720.render(cam, w7, h7, out=o7)
    torch.cuda.synchronize()
    t = time.perf_counter()
    V.image_quality(o7, r7)
    gpu_q = time.perf_counter() - t
    vol = inputs.make_volume(spec)
    t = time.perf_counter()
    cpu_dvr = inputs.generate_vdi(vol, cam, w7, h7, 1, spec["tf"], gamma=10.0).dvr
    t_dvr = time.perf_counter() - t
    del vol
    img = o7.cpu().numpy()
    t = time.perf_counter()
    Q.ssim(img, cpu_dvr)
    Q.psnr(img, cpu_dvr)
    t_q = time.perf_counter() - t
    res["gpu_vs_cpu_reference_720p_30deg"] = {
        "gpu_dvr_f64_ms": round(gpu_dvr, 3), "cpu_fp64_dvr_ms": round(1e3 * t_dvr, 1),
        "gpu_ssim_psnr_ms": round(1e3 * gpu_q, 3), "cpu_ssim_psnr_ms": round(1e3 * t_q, 1),
        "cpu_threads": inputs.generator_threads()}
    del dvol
    torch.cuda.empty_cache()
    log("quality 720p: " + ", ".join(f"{k} deg x{v['speedup_vs_dvr_f32']} vs DVR, SSIM {v['ssim']}" for k, v in row.items()))
    return res


def profile_generation(torch, V):
    import numpy as np

    import inputs
    a = torch.empty(2 ** 28, dtype=torch.float32, device="cuda").fill_(1.0)   # 1 GiB
    b = torch.empty_like(a)
    b.copy_(a)
    del a, b
    spec = inputs.WORKLOADS["720p"]
    vol = inputs.make_volume(spec)
    nz, ny, nx = vol.shape
    bmin, bmax = inputs.aabb_for((nx, ny, nz))
    dvol = torch.from_numpy(vol.view(np.int16)).cuda()
    for _ in range(2):
        V.generate(dvol, bmin, bmax, inputs.orbit_camera(0.0), spec["width"], spec["height"], spec["ns"], tf="knots4")
    torch.cuda.synchronize()
    log("generation profile pass done")


def generation_leg(src, torch, V):
    """GPU VDI generation (Section 3 with Alg. S1; the paper's Table 2 layout):
    mean time per VDI over 12 generating views 30 degrees apart, N_S = 15 / 20
    / 30, for the 720p and 1080p workloads' volumes, plus the N_S = 50 VDI the
    renderer is timed on, checked bit for bit against the CPU generator's."""
    import numpy as np

    import inputs
    res = {}
    for name in ("720p", "1080p"):
        spec = inputs.WORKLOADS[name]
        vol = inputs.make_volume(spec)
        nz, ny, nx = vol.shape
        bmin, bmax = inputs.aabb_for((nx, ny, nz))
        dvol = torch.from_numpy(vol.view(np.int16) if vol.dtype == np.uint16 else vol).cuda()
        del vol
        tf = {inputs.TF_RAMP: "ramp", inputs.TF_KNOTS4: "knots4"}[spec["tf"]]
        W0, H0 = spec["width"], spec["height"]
        row = {}
        for ns in (15, 20, 30):
            bufs = (torch.empty((H0, W0), dtype=torch.uint8, device="cuda"),
                    torch.empty((ns, H0, W0, 2), dtype=torch.float32, device="cuda"),
                    torch.empty((ns, H0, W0, 4), dtype=torch.float32, device="cuda"), None)
            V.generate(dvol, bmin, bmax, inputs.orbit_camera(0.0), W0, H0, ns, tf=tf, out=bufs)
            ms, segs = [], 0
            for k in range(12):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                V.generate(dvol, bmin, bmax, inputs.orbit_camera(30.0 * k), W0, H0, ns, tf=tf, out=bufs)
                e1.record()
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
                segs += int(bufs[0].sum())
            row[f"N_S={ns}"] = {"mean_ms": round(float(np.mean(ms)), 2), "max_ms": round(float(np.max(ms)), 2),
                                "supersegments_mean": segs // 12}
            del bufs
        if name == "720p":
            # The CPU FP64 generator (the oracle of this kernel) on the same VDI, on all host threads.
            vol = inputs.make_volume(spec)
            t = time.perf_counter()
            inputs.generate_vdi(vol, inputs.orbit_camera(0.0), W0, H0, 20, spec["tf"], 0.0)
            row["cpu_generator_N_S=20_view0_ms"] = round(1e3 * (time.perf_counter() - t), 1)
            row["cpu_generator_threads"] = inputs.generator_threads()
            del vol
        if name == "1080p":
            count, depth, rgba, _ = V.generate(dvol, bmin, bmax, src.camera, W0, H0, src.ns, tf=tf, gamma_out=False)
            torch.cuda.synchronize()
            same = (np.array_equal(count.cpu().numpy(), src.count) and np.array_equal(depth.cpu().numpy(), src.depth)
                    and np.array_equal(rgba.cpu().numpy(), src.rgba))
            row["N_S=50_bit_identical_to_cpu_generator"] = bool(same)
            # The generated planes straight into vdi_create (device to device, brick scatter, count grid).
            dv = V.DeviceVDI(count, depth, rgba, src.camera, src.bmin, src.bmax, grid_z=src.grid_z)
            torch.cuda.synchronize()
            t = time.perf_counter()
            hd = V.Vdi(dv)
            row["N_S=50_vdi_create_from_device_planes_ms"] = round(1e3 * (time.perf_counter() - t), 1)
            hd.close()
            del count, depth, rgba, dv
        del dvol
        torch.cuda.empty_cache()
        res[f"{name} ({nx}x{ny}x{nz} {'u16' if spec['volume'] == 'slab_u16' else 'f32'}, {W0}x{H0})"] = row
        log(f"generation {name}: " + ", ".join(f"{k} {v['mean_ms']} ms" for k, v in row.items() if isinstance(v, dict)))
    return res


def served_leg(torch, V):
    """The continuous-batching server against one request at a time."""
    from tests import harness
    return harness.serve_benchmark(log=log)


def cpu_baseline_leg(src, cams, per, precision, np, torch, V):
    """The FP64 oracle on the host cores, on a bounded random sample of the
    step's pixels; its per-frame time is extrapolated from the sample.  Also
    the accuracy of the FP32/FP16/BF16 GPU frames on the same sample."""
    import oracle
    rng = np.random.default_rng(1234)
    # The count grid once, untimed, as vdi_create builds it once outside the
    # timed step (the oracle would otherwise rebuild it for every preview
    # call, and the extrapolation would multiply that by the sample's inverse).
    grid = oracle.count_grid(src)
    frac = {1.0: 0.25, 2.0: 0.25, 4.0: 0.25}
    t_frames = 0.0
    n_px = 0
    errs = {"f32": [], "f16": [], "bf16": []}
    sq = {"f32": [0.0, 0], "f16": [0.0, 0], "bf16": [0.0, 0]}
    handles = {"f32": V.Vdi(src)}
    deq = {"f16": oracle.dequant_f16(src.rgba), "bf16": oracle.dequant_bf16(src.rgba)}
    for fmt in ("f16", "bf16"):
        handles[fmt] = V.Vdi(src, store=fmt)
    t_all = time.time()
    t_exact = 0.0
    for th in ANGLES:
        for (di, dr) in MODES:
            if dr == 0.0 and di == 1.0:
                n = max(64, int(frac[di] * W * H))
                pix = np.sort(rng.choice(W * H, size=n, replace=False))
                t = time.perf_counter()
                ref = oracle.render_exact(src, cams[th], W, H, pixels=pix)
                dt = time.perf_counter() - t
                flags = np.zeros(n, np.uint8)
                t_frames += dt / (n / (W * H))
                t_exact += dt / (n / (W * H))
            else:
                # A preview frame is its low-res ray grid (upsampling, negligible here, is not timed).
                w, hh = V.lowres_size(W, H, di)
                n = max(64, int(frac[di] * w * hh))
                tex = np.sort(rng.choice(w * hh, size=n, replace=False))
                t = time.perf_counter()
                oracle.render_preview(src, cams[th], w, hh, dr, pixels=tex, aspect=W / H, grid=grid)
                dt = time.perf_counter() - t
                t_frames += dt / (n / (w * hh))
            n_px += n
            if di == 1.0:
                ok = flags == 0
                for fmt, hh in handles.items():
                    img = hh.render(cams[th], W, H).cpu().numpy().reshape(-1, 4)[pix].astype(np.float64)
                    d = np.abs(img - ref)[ok]
                    errs[fmt].append(float(d.max()))
                    sq[fmt][0] += float((d ** 2).sum())
                    sq[fmt][1] += d.size
                    if fmt != "f32":
                        rq = oracle.render_exact(src, cams[th], W, H, pixels=pix, rgba=deq[fmt])
                        errs.setdefault(fmt + "_vs_dequantized", []).append(float(np.abs(img - rq).max()))
    for hh in handles.values():
        hh.close()
    cpu_s = time.time() - t_all
    mpix = len(per) * W * H / t_frames / 1e6
    mpix_exact = len(ANGLES) * W * H / t_exact / 1e6
    # One core: the exact frames at 0, 20 and 45 degrees on 0.2% of their pixels.
    t1, n1 = 0.0, 0
    for th in (0.0, 20.0, 45.0):
        pix = np.sort(rng.choice(W * H, size=int(0.002 * W * H), replace=False))
        t = time.perf_counter()
        oracle.render_exact(src, cams[th], W, H, pixels=pix, nthreads=1)
        t1 += time.perf_counter() - t
        n1 += len(pix)
    mpix_1 = n1 / t1 / 1e6
    cpu_model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    acc = {}
    for fmt in ("f32", "f16", "bf16"):
        mse = sq[fmt][0] / max(1, sq[fmt][1])
        acc[fmt] = {"max_abs_vs_fp64_oracle": errs[fmt] and max(errs[fmt]),
                    "psnr_db_vs_fp64_oracle": (None if mse == 0 else round(10 * math.log10(1.0 / mse), 2))}
        if fmt != "f32":
            acc[fmt]["max_abs_vs_oracle_on_dequantized"] = max(errs[fmt + "_vs_dequantized"])
    log(f"cpu baseline: {mpix:.4f} Mpixels/s extrapolated (exact frames {mpix_exact:.4f}), {n_px} rays in {cpu_s:.1f}s "
        f"on {oracle.threads()} threads ({cpu_model}); one thread, exact: {mpix_1:.4f} Mpixels/s")
    return {"value": round(mpix, 5), "unit": "Mpixels/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{n_px} random rays of the 30 frames of one step (25% of each exact frame's pixels, 25% of "
                      f"each preview frame's low-res ray grid), frame time extrapolated per frame; upsampling not "
                      f"timed",
            "exact_frames_Mpixels_per_s": round(mpix_exact, 5),
            "cpu_model": cpu_model,
            "single_core": {"Mpixels_per_s": round(mpix_1, 5),
                            "sample": f"exact frames at 0, 20, 45 deg, {n1} random pixels (0.2% of each), one thread"},
            "accuracy_exact_mode_sampled": acc, "host_seconds": round(cpu_s + t1, 1)}


if __name__ == "__main__":
    main()
