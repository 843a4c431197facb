"""Frame-time-paced preview rendering on the GPU (vdi_pace_* driving D_I
while D_R stays fixed).  On MI355X a preview frame's time depends only weakly
on D_I (it is bound by the longest rays' dependent loads, not by the number
of rays), so the test checks what the controller can do with that plant: it
keeps full resolution where the target is met, downsamples where it is not,
comes close to the target there, and returns to full resolution without
winding up."""
import sys

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


def test_paced_session_downsamples_only_where_needed():
    from paper_2206_08660_amd import vdi as V
    from paper_2206_08660_amd.pace import Pace
    from tests.harness import run_session
    src = inputs.load_workload("1080p", keep_dvr=False)
    W, H, d_r = 1920, 1080, 2.0
    easy, hard = inputs.orbit_camera(5.0), inputs.orbit_camera(40.0)
    with V.Vdi(src) as h:
        out = torch.empty((H, W, 4), dtype=torch.float32, device="cuda")
        fixed = lambda d: Pace(1e6, d_i_min=d, d_i_max=d, d_i_start=d)
        t_hard = float(np.median([t for _, t in run_session(h, [hard] * 12, W, H, d_r, fixed(1.0), out=out)][4:]))
        t_easy = float(np.median([t for _, t in run_session(h, [easy] * 12, W, H, d_r, fixed(1.0), out=out)][4:]))
        target = 0.85 * t_hard
        assert t_easy < 0.9 * target, (t_easy, target)
        with Pace(target, d_i_max=8.0) as p:
            log, kept = run_session(h, [easy] * 40 + [hard] * 80 + [easy] * 40, W, H, d_r, p, out=out,
                                    keep=(30, 119))
    d_i = np.array([d for d, _ in log])
    ms = np.array([t for _, t in log])
    rel = np.abs(ms[60:120] / target - 1.0)
    say(f"[gpu] target {target:.3f} ms (hard view at D_I=1: {t_hard:.3f}, easy: {t_easy:.3f}); hard phase: "
        f"D_I {d_i[60:120].mean():.2f}, |frame/target - 1| median {np.median(rel):.3f}; "
        f"easy again: D_I {d_i[150:].mean():.2f}")
    assert np.all(d_i[5:40] < 1.05)                 # target met at full resolution
    assert d_i[60:120].mean() > 1.2                  # downsampled where it was not
    assert np.median(rel) < 0.15
    assert d_i[150:].mean() < 1.3                    # back to full resolution, no windup
    # Paced frames are ordinary renders at the D_I the controller chose (a
    # fractional one in the hard phase): sampled pixels against the oracle,
    # on the pixels whose low-res texels rest on no tie.
    for k, cam in ((30, easy), (119, hard)):
        img = kept[k].cpu().numpy().astype(np.float64)
        pix = np.unique(np.concatenate([sample_pixels(W, H, 2000, seed=k), nonempty_stratum(img, 1000, seed=k)]))
        ref, flags = oracle.render_points(src, cam, W, H, float(d_i[k]), d_r, pix)
        ok = flags == 0
        say(f"[gpu] paced frame {k}: D_I {d_i[k]:.3f}, {int(ok.sum())} of {len(pix)} pixels off ties")
        assert ok.mean() > 0.9 and (ok & (ref[:, 3] > 0)).sum() >= 1000
        assert np.abs(img.reshape(-1, 4)[pix] - ref)[ok].max() <= TOL
