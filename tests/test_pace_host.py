"""The PI frame-time controller (vdi_pace_*) on model plants, on the host:
frame time a / D_I^2 + b (rays of a downsampled frame plus a fixed cost)."""
import math

import numpy as np
import pytest

from paper_2206_08660_amd import vdi as V
from paper_2206_08660_amd.pace import Pace


def plant(a, b):
    return lambda d_i: a / (d_i * d_i) + b


def run(pace, f, n, noise=0.0, rng=None):
    hist = []
    for _ in range(n):
        ms = f(pace.d_i)
        if noise:
            ms *= 1.0 + noise * rng.uniform(-1, 1)
        hist.append((pace.d_i, ms))
        pace.update(ms)
    return hist


def test_rejects_bad_arguments():
    import ctypes
    h = ctypes.c_void_p()
    L = V.lib()
    assert L.vdi_pace_create(0.0, 0.1, 0.3, 1.0, 8.0, 1.0, ctypes.byref(h)) == V.VDI_ERR_ARG
    assert L.vdi_pace_create(1.0, -0.1, 0.3, 1.0, 8.0, 1.0, ctypes.byref(h)) == V.VDI_ERR_ARG
    assert L.vdi_pace_create(1.0, 0.1, 0.3, 0.5, 8.0, 1.0, ctypes.byref(h)) == V.VDI_ERR_ARG
    assert L.vdi_pace_create(1.0, 0.1, 0.3, 2.0, 8.0, 1.0, ctypes.byref(h)) == V.VDI_ERR_ARG
    assert L.vdi_pace_create(1.0, 0.1, 0.3, 1.0, 8.0, 9.0, ctypes.byref(h)) == V.VDI_ERR_ARG
    assert L.vdi_pace_create(float("nan"), 0.1, 0.3, 1.0, 8.0, 1.0, ctypes.byref(h)) == V.VDI_ERR_ARG
    with Pace(1.0) as p:
        with pytest.raises(V.VdiError):
            p.update(0.0)
        with pytest.raises(V.VdiError):
            p.update(float("inf"))
    assert L.vdi_pace_destroy(None) == V.VDI_OK


def test_converges_on_a_ray_count_plant():
    f = plant(4.0, 0.05)  # 4.05 ms at D_I = 1
    with Pace(1.0) as p:
        h = run(p, f, 25)
    d_star = math.sqrt(4.0 / (1.0 - 0.05))
    assert abs(h[-1][0] - d_star) / d_star < 1e-3
    assert abs(h[-1][1] - 1.0) < 1e-3
    # no overshoot past the clamp, monotone approach in D_I on this plant
    assert all(1.0 <= d <= 8.0 for d, _ in h)


def test_follows_a_changing_plant():
    with Pace(1.0) as p:
        run(p, plant(4.0, 0.05), 25)
        h = run(p, plant(9.0, 0.05), 25)   # the view got harder
        assert abs(h[-1][1] - 1.0) < 1e-2
        h = run(p, plant(1.5, 0.05), 25)   # and easier again
        assert abs(h[-1][1] - 1.0) < 1e-2


def test_saturates_without_winding_up():
    # Unreachable target: D_I sits at its maximum ...
    with Pace(0.05, d_i_max=4.0) as p:
        h = run(p, plant(4.0, 0.2), 40)
        assert abs(h[-1][0] - 4.0) < 1e-6
        # ... and leaves it within a few frames once the target is reachable.
        h = run(p, plant(0.5, 0.01), 6)
        assert h[-1][0] < 4.0


def test_stays_at_full_resolution_when_fast_enough():
    with Pace(2.0) as p:
        h = run(p, plant(1.0, 0.1), 20)
    assert all(abs(d - 1.0) < 1e-6 for d, _ in h)


def test_holds_the_target_under_noise():
    rng = np.random.default_rng(5)
    with Pace(1.0) as p:
        h = run(p, plant(6.0, 0.1), 200, noise=0.05, rng=rng)
    err = np.array([ms for _, ms in h[20:]]) - 1.0
    assert np.mean(np.abs(err)) < 0.06 and np.percentile(np.abs(err), 95) < 0.15
