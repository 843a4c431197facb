"""Frame-time-paced preview rendering: binding of the vdi_pace_* calls of
include/vdi.h (a PI controller on the image downsampling D_I, Section 4.4 /
Section 5 of the paper) and a session loop that renders a camera path with it.
The frame time fed back is the GPU time of each render (HIP events on the
render stream)."""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

from . import vdi as V


class Pace:
    """PI controller on ln D_I holding a target frame time."""

    def __init__(self, target_ms: float, kp: float = 0.1, ki: float = 0.3, d_i_min: float = 1.0,
                 d_i_max: float = 8.0, d_i_start: Optional[float] = None):
        h = ctypes.c_void_p()
        start = d_i_min if d_i_start is None else d_i_start
        V._check(V.lib().vdi_pace_create(target_ms, kp, ki, d_i_min, d_i_max, start, ctypes.byref(h)))
        self._h = h
        self.d_i = float(start)

    def update(self, frame_ms: float) -> float:
        """Feed the last frame's time; returns the D_I for the next frame."""
        nd = ctypes.c_float()
        V._check(V.lib().vdi_pace_update(self._h, frame_ms, ctypes.byref(nd)))
        self.d_i = nd.value
        return self.d_i

    def close(self):
        if self._h is not None:
            h, self._h = self._h, None
            V._check(V.lib().vdi_pace_destroy(h))

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def run_session(vdi: "V.Vdi", cams: Sequence, width: int, height: int, d_r: float, pace: Pace, out=None,
                stream=None):
    """Render cams in order with D_I from `pace`; returns [(D_I, frame_ms)] per frame."""
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    if out is None:
        out = torch.empty((height, width, 4), dtype=torch.float32, device="cuda")
    log = []
    for cam in cams:
        d_i = pace.d_i
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        vdi.render(cam, width, height, d_i, d_r, out=out, stream=s)
        e1.record(s)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        log.append((d_i, ms))
        pace.update(ms)
    return log
