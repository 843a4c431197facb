"""Python binding of libvdi (include/vdi.h): argument marshalling only.

Every step of a render runs in the library's HIP kernels; torch provides the
device buffers and the stream.  Importing works without a GPU; any call that
needs the library raises if libvdi.so has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvdi.so")

VDI_OK = 0
VDI_ERR_ARG = -1
VDI_ERR_OOM = -2
VDI_ERR_HIP = -3
VDI_ERR_BUDGET = -4
VDI_ERR_STATE = -5

FORMATS = {"f32": 0, "f16": 1, "bf16": 2}
SEARCH = {"seeded": 0, "binary": 1, "linear": 2, "window": 3}

# Every symbol include/vdi.h declares.
EXPORTS = ("vdi_create", "vdi_render", "vdi_render_ex", "vdi_render_counters", "vdi_get_grid", "vdi_get_info",
           "vdi_destroy", "vdi_lowres_size", "vdi_plane_bytes", "vdi_last_error", "vdi_server_create",
           "vdi_server_submit", "vdi_server_poll", "vdi_server_drain", "vdi_server_get_stats",
           "vdi_server_reset_stats", "vdi_server_destroy", "vdi_replace_begin", "vdi_replace_poll",
           "vdi_pace_create", "vdi_pace_update", "vdi_pace_destroy", "vdi_generate", "vdi_dvr",
           "vdi_image_quality", "vdi_render_noalloc", "vdi_preview_counters", "vdi_server_submit_paced",
           "vdi_render_batch", "vdi_server_create_persistent")

VOXEL = {"f32": 0, "u16": 1}
TF = {"ramp": 0, "knots4": 1}
DVR_PRECISION = {"f64": 0, "f32": 1}


class VdiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libvdi error {code}: {msg}")
        self.code = code


class Camera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_float * 3), ("target", ctypes.c_float * 3), ("up", ctypes.c_float * 3),
                ("fov_y_deg", ctypes.c_float), ("near_plane", ctypes.c_float)]


class Desc(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("max_supersegments", ctypes.c_int32),
                ("camera_VO", Camera), ("aabb_min", ctypes.c_float * 3), ("aabb_max", ctypes.c_float * 3),
                ("count", ctypes.c_void_p), ("depth", ctypes.c_void_p), ("rgba", ctypes.c_void_p),
                ("rgba_fmt_in", ctypes.c_int32), ("rgba_fmt_store", ctypes.c_int32),
                ("grid_k", ctypes.c_int32), ("grid_nz", ctypes.c_int32), ("grid_z", ctypes.c_void_p),
                ("validate", ctypes.c_int32), ("planes_on_device", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("ess", ctypes.c_int32), ("search", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("max_supersegments", ctypes.c_int32),
                ("rgba_fmt", ctypes.c_int32), ("grid_k", ctypes.c_int32), ("grid_nz", ctypes.c_int32),
                ("grid_w", ctypes.c_int32), ("grid_h", ctypes.c_int32), ("device_bytes", ctypes.c_uint64),
                ("supersegments", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected_budget", ctypes.c_uint64), ("rejected_slots", ctypes.c_uint64),
                ("bytes_in_flight", ctypes.c_uint64), ("peak_bytes_in_flight", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("inflight", ctypes.c_int32), ("peak_inflight", ctypes.c_int32),
                ("queued", ctypes.c_int32), ("peak_batch", ctypes.c_int32),
                ("paced_completed", ctypes.c_uint64), ("deadlines_met", ctypes.c_uint64)]


class Volume(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("voxel_fmt", ctypes.c_int32), ("data", ctypes.c_void_p),
                ("aabb_min", ctypes.c_double * 3), ("aabb_max", ctypes.c_double * 3)]


class GenParams(ctypes.Structure):
    _fields_ = [("camera_VO", Camera), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("max_supersegments", ctypes.c_int32), ("tf", ctypes.c_int32), ("gamma", ctypes.c_double)]


class DvrParams(ctypes.Structure):
    _fields_ = [("camera", Camera), ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("tf", ctypes.c_int32),
                ("precision", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libvdi.so; raises if it was not built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2206_08660_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, F = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float
        L.vdi_create.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(P)]
        L.vdi_render.argtypes = [P, ctypes.POINTER(Camera), I32, I32, F, F, P, P]
        L.vdi_render_noalloc.argtypes = [P, ctypes.POINTER(Camera), I32, I32, F, F, P, P]
        L.vdi_render_batch.argtypes = [I32, P, P, P, P, P, P, P, P]
        L.vdi_render_ex.argtypes = [P, ctypes.POINTER(Camera), I32, I32, F, F, ctypes.POINTER(Opts), P, P]
        L.vdi_render_counters.argtypes = [P, ctypes.POINTER(Camera), I32, I32, ctypes.POINTER(Opts), P, P, P, P, P]
        L.vdi_preview_counters.argtypes = [P, ctypes.POINTER(Camera), I32, I32, F, F, P, P, P, P, P, P]
        L.vdi_get_grid.argtypes = [P, P, ctypes.c_size_t]
        L.vdi_get_info.argtypes = [P, ctypes.POINTER(Info)]
        L.vdi_destroy.argtypes = [P]
        L.vdi_replace_begin.argtypes = [P, ctypes.POINTER(Desc), P]
        L.vdi_replace_poll.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
        L.vdi_pace_create.argtypes = [F, F, F, F, F, F, ctypes.POINTER(P)]
        L.vdi_pace_update.argtypes = [P, F, ctypes.POINTER(F)]
        L.vdi_pace_destroy.argtypes = [P]
        L.vdi_lowres_size.argtypes = [I32, I32, F, ctypes.POINTER(I32), ctypes.POINTER(I32)]
        L.vdi_plane_bytes.argtypes = [I32, I32, I32, I32]
        L.vdi_plane_bytes.restype = ctypes.c_uint64
        L.vdi_last_error.restype = ctypes.c_char_p
        L.vdi_server_create.argtypes = [ctypes.c_uint64, I32, I32, ctypes.POINTER(P)]
        L.vdi_server_create_persistent.argtypes = [ctypes.c_uint64, I32, I32, ctypes.POINTER(P)]
        L.vdi_server_submit.argtypes = [P, P, ctypes.POINTER(Camera), I32, I32, F, F, P,
                                        ctypes.POINTER(ctypes.c_uint64)]
        L.vdi_server_submit_paced.argtypes = [P, P, ctypes.POINTER(Camera), I32, I32, P, F, P,
                                              ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(F)]
        L.vdi_server_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]
        L.vdi_server_drain.argtypes = [P]
        L.vdi_server_get_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
        L.vdi_server_reset_stats.argtypes = [P]
        L.vdi_server_destroy.argtypes = [P]
        L.vdi_generate.argtypes = [ctypes.POINTER(Volume), ctypes.POINTER(GenParams), P, P, P, P, P]
        L.vdi_dvr.argtypes = [ctypes.POINTER(Volume), ctypes.POINTER(DvrParams), P, P]
        L.vdi_image_quality.argtypes = [P, P, I32, I32, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double), P]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != VDI_OK:
        raise VdiError(rc, lib().vdi_last_error().decode())


def last_error() -> str:
    return lib().vdi_last_error().decode()


def camera(cam) -> Camera:
    """ctypes camera from any object with eye, target, up, fov_y_deg, near."""
    c = Camera()
    c.eye[:] = [float(x) for x in cam.eye]
    c.target[:] = [float(x) for x in cam.target]
    c.up[:] = [float(x) for x in cam.up]
    c.fov_y_deg = float(cam.fov_y_deg)
    c.near_plane = float(cam.near)
    return c


def lowres_size(width: int, height: int, d_i: float):
    w, h = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().vdi_lowres_size(width, height, d_i, ctypes.byref(w), ctypes.byref(h)))
    return w.value, h.value


def render_batch(frames, stream=None):
    """Render several frames in one call (vdi_render_batch).  `frames` is a
    sequence of (vdi, cam, width, height, d_i, d_r, out) with `out` a
    contiguous float32 CUDA tensor of height*width*4 elements each; the
    frames run on `stream` (default: torch's current stream)."""
    import torch
    n = len(frames)
    if n == 0:
        return
    vdis = (ctypes.c_void_p * n)()
    cams = (Camera * n)()
    ws, hs = (ctypes.c_int32 * n)(), (ctypes.c_int32 * n)()
    dis, drs = (ctypes.c_float * n)(), (ctypes.c_float * n)()
    outs = (ctypes.c_void_p * n)()
    for i, (v, cam, width, height, d_i, d_r, out) in enumerate(frames):
        if out.dtype != torch.float32 or not out.is_cuda or not out.is_contiguous() or \
                out.numel() < height * width * 4:
            raise ValueError(f"frame {i}: out must be a contiguous float32 CUDA tensor with height*width*4 elements")
        vdis[i] = v.handle
        cams[i] = camera(cam)
        ws[i], hs[i], dis[i], drs[i] = width, height, d_i, d_r
        outs[i] = out.data_ptr()
    _check(lib().vdi_render_batch(n, vdis, cams, ws, hs, dis, drs, outs, _stream_handle(stream)))


def plane_bytes(width: int, height: int, ns: int, fmt: str = "f32") -> int:
    return int(lib().vdi_plane_bytes(width, height, ns, FORMATS[fmt]))


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _opts(ess: bool, search: str) -> Opts:
    return Opts(1 if ess else 0, SEARCH[search])


def _on_device(a) -> bool:
    return bool(getattr(a, "is_cuda", False))


def _desc(src, store: str, validate: bool, rgba_in, fmt_in: str):
    """vdi_desc for src, and the arrays it points to (kept alive by the caller).
    Planes given as CUDA tensors are passed as device planes."""
    dev = _on_device(src.count)
    if dev:
        import torch
        count, depth = src.count, src.depth
        rgba = src.rgba if rgba_in is None else rgba_in
        ok = (_on_device(depth) and _on_device(rgba) and count.dtype == torch.uint8 and depth.dtype == torch.float32
              and rgba.dtype == (torch.float32 if fmt_in == "f32" else rgba.dtype)
              and all(t.is_contiguous() for t in (count, depth, rgba)))
        if not ok:
            raise ValueError("device planes must be contiguous CUDA tensors: count uint8, depth float32, rgba float32 "
                             "(or 16-bit with fmt_in)")
        ptr = lambda t: t.data_ptr()
    else:
        count = np.ascontiguousarray(src.count, dtype=np.uint8)
        depth = np.ascontiguousarray(src.depth, dtype=np.float32)
        rgba = np.ascontiguousarray(src.rgba if rgba_in is None else rgba_in)
        if fmt_in == "f32":
            rgba = rgba.astype(np.float32, copy=False)
        ptr = lambda a: a.ctypes.data
    gz = None if src.grid_z is None else np.ascontiguousarray(src.grid_z, dtype=np.float32)
    d = Desc()
    d.width, d.height, d.max_supersegments = src.width, src.height, src.ns
    d.camera_VO = camera(src.camera)
    d.aabb_min[:] = [float(x) for x in src.bmin]
    d.aabb_max[:] = [float(x) for x in src.bmax]
    d.count = ptr(count)
    d.depth = ptr(depth)
    d.rgba = ptr(rgba)
    d.rgba_fmt_in = FORMATS[fmt_in]
    d.rgba_fmt_store = FORMATS[store]
    d.grid_k, d.grid_nz = src.grid_k, src.grid_nz
    d.grid_z = None if gz is None else gz.ctypes.data
    d.validate = 1 if validate else 0
    d.planes_on_device = 1 if dev else 0
    return d, (count, depth, rgba, gz)


class DeviceVDI:
    """A VDI whose planes are CUDA tensors in the vdi_desc layout (as
    vdi_generate writes them); Vdi() and Vdi.replace_begin() take it without a
    copy through host memory."""

    def __init__(self, count, depth, rgba, camera, bmin, bmax, grid_k: int = 8, grid_nz: int = 20, grid_z=None):
        self.count, self.depth, self.rgba = count, depth, rgba
        self.ns, self.height, self.width = int(depth.shape[0]), int(depth.shape[1]), int(depth.shape[2])
        self.camera, self.bmin, self.bmax = camera, tuple(bmin), tuple(bmax)
        self.grid_k, self.grid_nz, self.grid_z = grid_k, grid_nz, grid_z


class Vdi:
    """A VDI resident in device memory (vdi_create ... vdi_destroy)."""

    def __init__(self, src, store: str = "f32", validate: bool = False, rgba_in: Optional[np.ndarray] = None,
                 fmt_in: str = "f32"):
        """src: any object with width, height, ns, camera, bmin, bmax, count,
        depth, rgba, grid_k, grid_nz, grid_z (e.g. inputs.VDI)."""
        self._h = None
        d, _keep = _desc(src, store, validate, rgba_in, fmt_in)
        if d.planes_on_device:
            import torch
            torch.cuda.current_stream().synchronize()   # the planes may still be written there
        h = ctypes.c_void_p()
        _check(lib().vdi_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self.width, self.height, self.ns, self.store = src.width, src.height, src.ns, store

    def replace_begin(self, src, stream=None, validate: bool = False, rgba_in: Optional[np.ndarray] = None,
                      fmt_in: str = "f32"):
        """Start uploading another VDI of the same shape (vdi_replace_begin),
        after the work enqueued on `stream` (default: torch's current stream)."""
        d, _keep = _desc(src, self.store, validate, rgba_in, fmt_in)
        _check(lib().vdi_replace_begin(self.handle, ctypes.byref(d), _stream_handle(stream)))

    def replace_poll(self) -> bool:
        """True once the replacement has been swapped in (vdi_replace_poll)."""
        sw = ctypes.c_int32()
        _check(lib().vdi_replace_poll(self.handle, ctypes.byref(sw)))
        return bool(sw.value)

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise VdiError(VDI_ERR_STATE, "VDI already destroyed")
        return self._h

    def render(self, cam, width: int, height: int, d_i: float = 1.0, d_r: float = 0.0, out=None, stream=None,
               ess: bool = True, search: str = "window"):
        """Render into a float32 [height, width, 4] device tensor (allocated if
        `out` is None) on `stream` (default: torch's current stream)."""
        import torch
        if out is None:
            out = torch.empty((height, width, 4), dtype=torch.float32, device="cuda")
        if out.dtype != torch.float32 or not out.is_cuda or not out.is_contiguous() or out.numel() < height * width * 4:
            raise ValueError("out must be a contiguous float32 CUDA tensor with height*width*4 elements")
        c = camera(cam)
        o = _opts(ess, search)
        _check(lib().vdi_render_ex(self.handle, ctypes.byref(c), width, height, d_i, d_r, ctypes.byref(o),
                                   ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out

    def render_noalloc(self, cam, width: int, height: int, d_i: float = 1.0, d_r: float = 0.0, out=None,
                       stream=None):
        """vdi_render_noalloc: the vdi_render image, with the low-res image of a
        downsampled render in the library's static device scratch (no device
        allocation by the library).  `out` as in render()."""
        import torch
        if out is None:
            out = torch.empty((height, width, 4), dtype=torch.float32, device="cuda")
        if out.dtype != torch.float32 or not out.is_cuda or not out.is_contiguous() or out.numel() < height * width * 4:
            raise ValueError("out must be a contiguous float32 CUDA tensor with height*width*4 elements")
        c = camera(cam)
        _check(lib().vdi_render_noalloc(self.handle, ctypes.byref(c), width, height, d_i, d_r,
                                        ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out

    def preview_counters(self, cam, width: int, height: int, d_i: float, d_r: float, stream=None):
        """Instrumented preview of the low-res ray grid (vdi_preview_counters):
        (low-res image [h, w, 4], touched_lists [H_O, W_O] u8, touched_slots
        [N_S, H_O, W_O] u8, touched_cells [N_z, GH, GW] u8, ray_stats [h, w, 2]
        i32), all torch CUDA tensors."""
        import torch
        w, h = lowres_size(width, height, d_i)
        inf = self.info()
        out = torch.empty((h, w, 4), dtype=torch.float32, device="cuda")
        tl = torch.zeros((self.height, self.width), dtype=torch.uint8, device="cuda")
        ts = torch.zeros((self.ns, self.height, self.width), dtype=torch.uint8, device="cuda")
        tc = torch.zeros((inf.grid_nz, inf.grid_h, inf.grid_w), dtype=torch.uint8, device="cuda")
        st = torch.zeros((h, w, 2), dtype=torch.int32, device="cuda")
        c = camera(cam)
        _check(lib().vdi_preview_counters(self.handle, ctypes.byref(c), width, height, d_i, d_r,
                                          ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(tl.data_ptr()),
                                          ctypes.c_void_p(ts.data_ptr()), ctypes.c_void_p(tc.data_ptr()),
                                          ctypes.c_void_p(st.data_ptr()), _stream_handle(stream)))
        return out, tl, ts, tc, st

    def render_counters(self, cam, width: int, height: int, ess: bool = False, search: str = "window",
                        stream=None):
        """Instrumented exact render: (image, touched_lists [H_O, W_O] u8,
        touched_slots [N_S, H_O, W_O] u8, ray_stats [H, W, 2] i32), all torch CUDA tensors."""
        import torch
        out = torch.empty((height, width, 4), dtype=torch.float32, device="cuda")
        tl = torch.zeros((self.height, self.width), dtype=torch.uint8, device="cuda")
        ts = torch.zeros((self.ns, self.height, self.width), dtype=torch.uint8, device="cuda")
        st = torch.zeros((height, width, 2), dtype=torch.int32, device="cuda")
        c = camera(cam)
        o = _opts(ess, search)
        _check(lib().vdi_render_counters(self.handle, ctypes.byref(c), width, height, ctypes.byref(o),
                                         ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(tl.data_ptr()),
                                         ctypes.c_void_p(ts.data_ptr()), ctypes.c_void_p(st.data_ptr()),
                                         _stream_handle(stream)))
        return out, tl, ts, st

    def info(self) -> Info:
        i = Info()
        _check(lib().vdi_get_info(self.handle, ctypes.byref(i)))
        return i

    def grid(self) -> np.ndarray:
        i = self.info()
        g = np.zeros((i.grid_nz, i.grid_h, i.grid_w), dtype=np.uint32)
        _check(lib().vdi_get_grid(self.handle, ctypes.c_void_p(g.ctypes.data), g.size))
        return g

    def close(self):
        if self._h is not None:
            h, self._h = self._h, None
            _check(lib().vdi_destroy(h))

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _volume(volume, aabb_min, aabb_max) -> Volume:
    import torch
    if volume.dim() != 3 or not volume.is_cuda or not volume.is_contiguous():
        raise ValueError("volume must be a contiguous 3-d device tensor [nz, ny, nx]")
    if volume.dtype == torch.float32:
        fmt = VOXEL["f32"]
    elif volume.dtype in (torch.int16, getattr(torch, "uint16", torch.int16)):
        fmt = VOXEL["u16"]
    else:
        raise TypeError("volume must be float32 or 16-bit")
    nz, ny, nx = volume.shape
    v = Volume(nx, ny, nz, fmt, ctypes.c_void_p(volume.data_ptr()))
    v.aabb_min[:] = [float(x) for x in aabb_min]
    v.aabb_max[:] = [float(x) for x in aabb_max]
    return v


def dvr(volume, aabb_min, aabb_max, cam, width: int, height: int, tf: str = "knots4", precision: str = "f64",
        out=None, stream=None):
    """vdi_dvr: direct volume rendering of a device volume; returns the
    [height, width, 4] float32 device image (the vdi_render layout)."""
    import torch
    v = _volume(volume, aabb_min, aabb_max)
    p = DvrParams()
    p.camera = camera(cam)
    p.width, p.height, p.tf, p.precision = width, height, TF[tf], DVR_PRECISION[precision]
    if out is None:
        out = torch.empty((height, width, 4), dtype=torch.float32, device=volume.device)
    elif tuple(out.shape) != (height, width, 4) or out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 [height, width, 4] tensor")
    _check(lib().vdi_dvr(ctypes.byref(v), ctypes.byref(p), ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def image_quality(image, reference, stream=None):
    """vdi_image_quality: (SSIM, PSNR) of a device RGBA float32 image against a reference."""
    import torch
    for t in (image, reference):
        if t.dim() != 3 or t.shape[2] != 4 or t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("images must be contiguous float32 [height, width, 4] device tensors")
    if image.shape != reference.shape:
        raise ValueError("images differ in shape")
    s, p = ctypes.c_double(), ctypes.c_double()
    _check(lib().vdi_image_quality(ctypes.c_void_p(image.data_ptr()), ctypes.c_void_p(reference.data_ptr()),
                                   image.shape[1], image.shape[0], ctypes.byref(s), ctypes.byref(p),
                                   _stream_handle(stream)))
    return s.value, p.value


def generate(volume, aabb_min, aabb_max, cam, width: int, height: int, ns: int, tf: str = "knots4",
             gamma: float = 0.0, out=None, gamma_out: bool = True, stream=None):
    """vdi_generate: a VDI from a device volume ([nz, ny, nx] float32, or
    uint16 / int16 holding uint16 bits), as device tensors in the vdi_desc
    layout: (count [H, W] uint8, depth [NS, H, W, 2] f32, rgba [NS, H, W, 4]
    f32, gamma [H, W] f64 or None).  `out` may give those tensors to fill."""
    import torch
    v = _volume(volume, aabb_min, aabb_max)
    p = GenParams()
    p.camera_VO = camera(cam)
    p.width, p.height, p.max_supersegments, p.tf, p.gamma = width, height, ns, TF[tf], float(gamma)
    dev = volume.device
    if out is None:
        count = torch.empty((height, width), dtype=torch.uint8, device=dev)
        depth = torch.empty((ns, height, width, 2), dtype=torch.float32, device=dev)
        rgba = torch.empty((ns, height, width, 4), dtype=torch.float32, device=dev)
        gam = torch.empty((height, width), dtype=torch.float64, device=dev) if gamma_out else None
    else:
        count, depth, rgba, gam = out
        if (tuple(count.shape) != (height, width) or count.dtype != torch.uint8
                or tuple(depth.shape) != (ns, height, width, 2) or depth.dtype != torch.float32
                or tuple(rgba.shape) != (ns, height, width, 4) or rgba.dtype != torch.float32
                or (gam is not None and (tuple(gam.shape) != (height, width) or gam.dtype != torch.float64))
                or not all(t.is_contiguous() and t.is_cuda for t in (count, depth, rgba))):
            raise ValueError("output tensors do not match the VDI shape")
    _check(lib().vdi_generate(ctypes.byref(v), ctypes.byref(p), ctypes.c_void_p(count.data_ptr()),
                              ctypes.c_void_p(depth.data_ptr()), ctypes.c_void_p(rgba.data_ptr()),
                              None if gam is None else ctypes.c_void_p(gam.data_ptr()), _stream_handle(stream)))
    return count, depth, rgba, gam
