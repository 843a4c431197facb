"""Served form: binding of the vdi_server_* calls of include/vdi.h
(continuous batching of VDI render requests, admission by request slots and
a device-memory budget)."""
from __future__ import annotations

import ctypes
from typing import Optional

from . import vdi as V


class Server:
    """A continuous-batching server on the current device: batched launches
    (vdi_server_create), or one persistent kernel when `persistent` is set
    (vdi_server_create_persistent; `waves_per_simd` 0 = as many as fit)."""

    def __init__(self, budget_bytes: int, max_inflight: int = 64, streams: int = 0, persistent: bool = False,
                 waves_per_simd: int = 0):
        h = ctypes.c_void_p()
        if persistent:
            V._check(V.lib().vdi_server_create_persistent(int(budget_bytes), int(max_inflight), int(waves_per_simd),
                                                          ctypes.byref(h)))
        else:
            V._check(V.lib().vdi_server_create(int(budget_bytes), int(max_inflight), int(streams), ctypes.byref(h)))
        self._h = h

    def submit(self, vdi: "V.Vdi", cam, width: int, height: int, d_i: float, d_r: float, out) -> Optional[int]:
        """Ticket, or None when the request does not fit the budget or slots now."""
        c = V.camera(cam)
        t = ctypes.c_uint64()
        rc = V.lib().vdi_server_submit(self._h, vdi.handle, ctypes.byref(c), width, height, d_i, d_r,
                                       ctypes.c_void_p(out.data_ptr()), ctypes.byref(t))
        if rc == V.VDI_ERR_BUDGET:
            return None
        V._check(rc)
        return t.value

    def submit_paced(self, vdi: "V.Vdi", cam, width: int, height: int, session, d_r: float, out):
        """A request of a paced session (vdi_server_submit_paced): (ticket,
        D_I used), or None when it does not fit the budget or slots now.
        `session` is a pace.Pace whose controller the server feeds."""
        c = V.camera(cam)
        t = ctypes.c_uint64()
        d_i = ctypes.c_float()
        rc = V.lib().vdi_server_submit_paced(self._h, vdi.handle, ctypes.byref(c), width, height, session.handle,
                                             d_r, ctypes.c_void_p(out.data_ptr()), ctypes.byref(t), ctypes.byref(d_i))
        if rc == V.VDI_ERR_BUDGET:
            return None
        V._check(rc)
        return t.value, d_i.value

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int()
        V._check(V.lib().vdi_server_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(d)))
        return bool(d.value)

    def drain(self):
        V._check(V.lib().vdi_server_drain(self._h))

    def stats(self) -> dict:
        s = V.ServerStats()
        V._check(V.lib().vdi_server_get_stats(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in V.ServerStats._fields_}

    def reset_stats(self):
        V._check(V.lib().vdi_server_reset_stats(self._h))

    def close(self):
        if self._h is not None:
            h, self._h = self._h, None
            V._check(V.lib().vdi_server_destroy(h))

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
