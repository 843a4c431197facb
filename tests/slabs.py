"""Layered volumes with closed-form generation results (paper Section 3,
Eq. 1; supplement Alg. S1), for pins of the VDI generators that do not go
through either generator.

A 32^3 float32 volume of constant layers along z, seen from the generating
view V_O (eye at (0, 0, 1.5) looking down -z) at 33 x 33: the centre pixel's
ray runs along the volume's axis through x = y = 0, enters at depth 1.0,
leaves at 2.0, and takes one sample per voxel layer, each at a layer's centre
(one voxel long, so its corrected opacity is the transfer function's own).
Interpolation in x and y is between equal values, so every sample is exactly
its layer's value.  With the ramp transfer function, RGB = (v, 0.25 + 0.5 v,
1 - v) and alpha = 0.2 (v - 0.05) / 0.95.
"""
import math

import numpy as np

import inputs

N = 32
W = H = 33
CX = CY = 16


def ramp(v: float):
    c = np.array([v, 0.25 + 0.5 * v, 1.0 - v])
    a = 0.2 * min(max((v - 0.05) / 0.95, 0.0), 1.0)
    return c, a


def volume(layers):
    """layers: (value, count) pairs in the order the ray meets them (from
    z = +0.5 downwards), counts summing to 32."""
    assert sum(n for _, n in layers) == N
    vol = np.zeros((N, N, N), np.float32)
    k = N
    for v, n in layers:
        vol[k - n:k] = v
        k -= n
    return vol


def run(layers):
    """(colour, opacity, samples) of each layer's merged run: the front-to-back
    composite of n samples of one value is that value's colour with opacity
    1 - (1 - a)^n."""
    out = []
    for v, n in layers:
        c, a = ramp(v)
        out.append((c, 1.0 - (1.0 - a) ** n, n))
    return out


def merge(runs):
    """Straight colour and accumulated opacity of consecutive runs merged
    into one supersegment (front to back), and their sample count."""
    acc, T, n = np.zeros(3), 1.0, 0
    for c, a, k in runs:
        acc += T * a * c
        T *= 1.0 - a
        n += k
    alpha = 1.0 - T
    return acc / alpha, alpha, n


def eq1_distance(open_runs, nxt):
    """Eq. 1 distance between the open supersegment made of `open_runs` and
    the next sample, whose value starts run `nxt`: the open one's colour
    times its opacity normalised to one sample, against the sample's colour
    times its opacity (the reading under which a constant run never splits)."""
    C, alpha, n = merge(open_runs)
    abar = 1.0 - (1.0 - alpha) ** (1.0 / n)
    c, a = ramp(nxt)
    return float(np.linalg.norm(C * abar - c * a))


def depth_bounds(layers):
    """V_O depths of the layer boundaries on the centre ray: 1.0 + k / 32."""
    b, k = [1.0], 0
    for _, n in layers:
        k += n
        b.append(1.0 + k / N)
    return b


def camera():
    return inputs.orbit_camera(0.0)


def expected(layers, gamma: float, ns: int):
    """Supersegments of the centre ray at sensitivity gamma, capped at ns:
    [(front, back, colour, opacity)].  A supersegment closes before a sample
    whose Eq. 1 distance from it reaches gamma; samples of one layer are equal,
    so only a layer's first sample can close one, unless the open one mixes
    layers, where every sample of the layer is checked.  With ns - 1 closed,
    the last takes every remaining sample."""
    runs = run(layers)
    bounds = depth_bounds(layers)
    segs = []          # closed: list of (first run, last run)
    start = 0
    for i in range(1, len(layers)):
        if len(segs) == ns - 1:
            break
        if eq1_distance(runs[start:i], layers[i][0]) >= gamma:
            segs.append((start, i - 1))
            start = i
            continue
        # merged into the open supersegment: check the rest of the layer's samples
        c, a = ramp(layers[i][0])
        for k in range(1, layers[i][1]):
            part = (c, 1.0 - (1.0 - a) ** k, k)
            assert eq1_distance(runs[start:i] + [part], layers[i][0]) < gamma, "split inside a layer"
    segs.append((start, len(layers) - 1))
    out = []
    for s, e in segs:
        C, alpha, _ = merge(runs[s:e + 1])
        out.append((bounds[s], bounds[e + 1], C, alpha))
    return out


def check(vdi_count, vdi_depth, vdi_rgba, want, tol=2e-6):
    """The centre list of generated planes (count [H, W], depth [NS, H, W, 2],
    rgba [NS, H, W, 4]) against `expected`."""
    assert int(vdi_count[CY, CX]) == len(want), (int(vdi_count[CY, CX]), len(want))
    for j, (f, b, C, a) in enumerate(want):
        assert vdi_depth[j, CY, CX, 0] == np.float32(f) and vdi_depth[j, CY, CX, 1] == np.float32(b), j
        assert np.abs(vdi_rgba[j, CY, CX, :3] - C).max() <= tol and abs(vdi_rgba[j, CY, CX, 3] - a) <= tol, j


TWO = [(0.8, 16), (0.3, 16)]
THREE = [(0.8, 8), (0.5, 8), (0.2, 16)]
# Centre-ray counts of THREE against gamma: splits a|b below d(a, b) = 0.0977,
# b|c below d(b, c) = 0.0591, and the merged a+b | c below 0.1126.
THREE_CASES = [(0.05, 3), (0.08, 2), (0.105, 2), (0.2, 1)]


def searched_gamma_three():
    """The bracket search on THREE with N_S = 2 (delta = 0): 1e-5 gives 3
    supersegments; the midpoints lo + D/2, D/4, D/8 (D = sqrt 3 - 1e-5) give 1;
    lo + D/16 = 0.108 lies in [0.0977, 0.1126) and gives 2, which stands."""
    return 1e-5 + (math.sqrt(3.0) - 1e-5) / 16.0
