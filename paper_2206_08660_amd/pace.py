"""Frame-time-paced preview rendering: binding of the vdi_pace_* calls of
include/vdi.h (a PI controller on the image downsampling D_I, Section 4.4 /
Section 5 of the paper)."""
from __future__ import annotations

import ctypes
from typing import Optional

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

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise V.VdiError(V.VDI_ERR_STATE, "pace controller already destroyed")
        return self._h

    def close(self):
        if self._h is not None:
            h, self._h = self._h, None
            V._check(V.lib().vdi_pace_destroy(h))

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
