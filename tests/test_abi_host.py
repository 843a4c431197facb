"""The C ABI on the host: the library loads, exports every symbol the header
declares, and its host-only calls and argument checks work without a GPU."""
import ctypes
import os
import re

import pytest

from paper_2206_08660_amd import vdi as V

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "vdi.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(vdi_[a-z_0-9]+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = V.lib()
    names = _header_functions()
    assert len(names) >= 15
    assert set(names) == set(V.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_plane_bytes_match_paper_sizes():
    # Section 6.3 / 6.1: RGBA32F colour + R32F front/back depth per slot.
    mib = lambda b: b / 2 ** 20
    for (w, h, want) in [(1280, 720, 422), (1920, 1080, 950), (1024, 1024, 480)]:
        b = V.plane_bytes(w, h, 20, "f32") - w * h   # without the count plane
        assert abs(mib(b) - want) < 1.0
    assert V.plane_bytes(1920, 1080, 50, "f16") - 1920 * 1080 == 1920 * 1080 * 50 * 16


def test_lowres_size():
    assert V.lowres_size(1920, 1080, 2.0) == (960, 540)
    assert V.lowres_size(1920, 1080, 4.0) == (480, 270)
    assert V.lowres_size(1280, 720, 3.0) == (427, 240)
    assert V.lowres_size(7, 5, 1000.0) == (1, 1)
    with pytest.raises(V.VdiError):
        V.lowres_size(10, 10, 0.5)


def test_render_rejects_bad_arguments_before_any_device_work():
    lib = V.lib()
    cam = V.Camera()
    out = ctypes.c_void_p(16)
    assert lib.vdi_render(None, ctypes.byref(cam), 4, 4, 1.0, 0.0, out, None) == V.VDI_ERR_ARG
    assert "null" in V.last_error()
    fake = ctypes.c_void_p(1)   # never dereferenced: argument checks come first
    assert lib.vdi_render(fake, None, 4, 4, 1.0, 0.0, out, None) == V.VDI_ERR_ARG
    assert lib.vdi_render(fake, ctypes.byref(cam), 0, 4, 1.0, 0.0, out, None) == V.VDI_ERR_ARG
    assert lib.vdi_render(fake, ctypes.byref(cam), 4, 4, 0.5, 0.0, out, None) == V.VDI_ERR_ARG
    assert lib.vdi_render(fake, ctypes.byref(cam), 4, 4, 1.0, -1.0, out, None) == V.VDI_ERR_ARG
    assert lib.vdi_render(fake, ctypes.byref(cam), 4, 4, float("nan"), 0.0, out, None) == V.VDI_ERR_ARG
    assert lib.vdi_render(fake, ctypes.byref(cam), 4, 4, 1.0, 0.0, None, None) == V.VDI_ERR_ARG


def test_render_batch_rejects_bad_arguments_before_any_device_work():
    lib = V.lib()
    n = 2
    vdis = (ctypes.c_void_p * n)(None, None)
    cams = (V.Camera * n)()
    ws, hs = (ctypes.c_int32 * n)(4, 4), (ctypes.c_int32 * n)(4, 4)
    dis, drs = (ctypes.c_float * n)(1.0, 1.0), (ctypes.c_float * n)(0.0, 0.0)
    outs = (ctypes.c_void_p * n)(16, 4096)
    for bad_n in (0, -1, 1025):
        assert lib.vdi_render_batch(bad_n, vdis, cams, ws, hs, dis, drs, outs, None) == V.VDI_ERR_ARG
    assert lib.vdi_render_batch(n, None, cams, ws, hs, dis, drs, outs, None) == V.VDI_ERR_ARG
    assert lib.vdi_render_batch(n, vdis, cams, ws, hs, dis, drs, None, None) == V.VDI_ERR_ARG
    assert lib.vdi_render_batch(n, vdis, cams, ws, hs, dis, drs, outs, None) == V.VDI_ERR_ARG
    assert "frame 0" in V.last_error() and "null" in V.last_error()
    vdis[0] = 1   # never dereferenced: frame 0's other arguments are checked first
    ws[0] = 0
    assert lib.vdi_render_batch(n, vdis, cams, ws, hs, dis, drs, outs, None) == V.VDI_ERR_ARG
    assert "frame 0" in V.last_error()


def test_create_rejects_bad_descriptors_before_any_device_work():
    lib = V.lib()
    h = ctypes.c_void_p()
    assert lib.vdi_create(None, ctypes.byref(h)) == V.VDI_ERR_ARG
    d = V.Desc()
    d.width, d.height, d.max_supersegments = 4, 4, 0
    assert lib.vdi_create(ctypes.byref(d), ctypes.byref(h)) == V.VDI_ERR_ARG
    d.max_supersegments = 300
    assert lib.vdi_create(ctypes.byref(d), ctypes.byref(h)) == V.VDI_ERR_ARG
    d.max_supersegments = 4
    assert lib.vdi_create(ctypes.byref(d), ctypes.byref(h)) == V.VDI_ERR_ARG   # null planes
    assert h.value is None


def test_destroy_null_is_noop():
    assert V.lib().vdi_destroy(None) == V.VDI_OK


def test_create_rejects_count_grid_of_2_31_cells():
    lib = V.lib()
    h = ctypes.c_void_p()
    d = V.Desc()
    d.width, d.height, d.max_supersegments = 32768, 32768, 4
    fake = 16   # never dereferenced: the grid shape is checked before the planes are read
    d.count, d.depth, d.rgba = fake, fake, fake
    d.grid_k, d.grid_nz = 1, 2          # 2 * 2^30 = 2^31 cells
    assert lib.vdi_create(ctypes.byref(d), ctypes.byref(h)) == V.VDI_ERR_ARG
    assert "2^31" in V.last_error()


def test_server_create_rejects_bad_arguments_before_any_device_work():
    lib = V.lib()
    h = ctypes.c_void_p()
    assert lib.vdi_server_create(1 << 30, 4, 0, None) == V.VDI_ERR_ARG
    assert lib.vdi_server_create(0, 4, 0, ctypes.byref(h)) == V.VDI_ERR_ARG
    assert lib.vdi_server_create(1 << 30, 0, 0, ctypes.byref(h)) == V.VDI_ERR_ARG
    assert lib.vdi_server_create(1 << 30, 4097, 0, ctypes.byref(h)) == V.VDI_ERR_ARG
    assert lib.vdi_server_create(1 << 30, 4, -1, ctypes.byref(h)) == V.VDI_ERR_ARG
    assert lib.vdi_server_create(1 << 30, 4, 9, ctypes.byref(h)) == V.VDI_ERR_ARG
    assert "streams" in V.last_error()
    assert h.value is None
    assert lib.vdi_server_destroy(None) == V.VDI_OK


def test_persistent_server_create_rejects_bad_arguments_before_any_device_work():
    lib = V.lib()
    h = ctypes.c_void_p()
    assert lib.vdi_server_create_persistent(1 << 30, 4, 0, None) == V.VDI_ERR_ARG
    assert lib.vdi_server_create_persistent(0, 4, 0, ctypes.byref(h)) == V.VDI_ERR_ARG
    assert lib.vdi_server_create_persistent(1 << 30, 0, 0, ctypes.byref(h)) == V.VDI_ERR_ARG
    assert lib.vdi_server_create_persistent(1 << 30, 4097, 0, ctypes.byref(h)) == V.VDI_ERR_ARG
    assert lib.vdi_server_create_persistent(1 << 30, 4, -1, ctypes.byref(h)) == V.VDI_ERR_ARG
    assert lib.vdi_server_create_persistent(1 << 30, 4, 17, ctypes.byref(h)) == V.VDI_ERR_ARG
    assert "waves_per_simd" in V.last_error()
    assert h.value is None


def test_replace_rejects_null_arguments_before_any_device_work():
    lib = V.lib()
    d = V.Desc()
    assert lib.vdi_replace_begin(None, ctypes.byref(d), None) == V.VDI_ERR_ARG
    assert lib.vdi_replace_begin(ctypes.c_void_p(1), None, None) == V.VDI_ERR_ARG
    sw = ctypes.c_int32(7)
    assert lib.vdi_replace_poll(None, ctypes.byref(sw)) == V.VDI_ERR_ARG
    assert lib.vdi_replace_poll(ctypes.c_void_p(1), None) == V.VDI_ERR_ARG


def test_generate_rejects_bad_arguments_before_any_device_work():
    lib = V.lib()
    buf = ctypes.c_void_p(16)  # never dereferenced: every case fails its checks first

    def good():
        v = V.Volume(8, 8, 8, V.VOXEL["f32"], buf)
        v.aabb_min[:] = [-0.5] * 3
        v.aabb_max[:] = [0.5] * 3
        p = V.GenParams()
        c = V.Camera()
        c.eye[:] = [0.0, 0.0, 1.5]
        c.target[:] = [0.0, 0.0, 0.0]
        c.up[:] = [0.0, 1.0, 0.0]
        c.fov_y_deg, c.near_plane = 50.0, 0.1
        p.camera_VO = c
        p.width, p.height, p.max_supersegments, p.tf, p.gamma = 16, 16, 4, V.TF["ramp"], 0.0
        return v, p

    def call(v, p, outs=(buf, buf, buf)):
        return lib.vdi_generate(None if v is None else ctypes.byref(v), None if p is None else ctypes.byref(p),
                                *outs, None, None)

    v, p = good()
    assert call(None, p) == V.VDI_ERR_ARG
    assert call(v, None) == V.VDI_ERR_ARG
    assert call(v, p, (buf, None, buf)) == V.VDI_ERR_ARG
    cases = [
        ("nx", lambda v, p: setattr(v, "nx", 0), "volume size"),
        ("fmt", lambda v, p: setattr(v, "voxel_fmt", 5), "voxel format"),
        ("aabb", lambda v, p: v.aabb_max.__setitem__(1, -0.5), "AABB"),
        ("nan aabb", lambda v, p: v.aabb_min.__setitem__(0, float("nan")), "AABB"),
        ("width", lambda v, p: setattr(p, "width", 0), "VDI size"),
        ("ns", lambda v, p: setattr(p, "max_supersegments", 256), "max_supersegments"),
        ("tf", lambda v, p: setattr(p, "tf", 9), "transfer function"),
        ("gamma", lambda v, p: setattr(p, "gamma", -1.0), "gamma"),
        ("gamma nan", lambda v, p: setattr(p, "gamma", float("nan")), "gamma"),
        ("fov", lambda v, p: setattr(p.camera_VO, "fov_y_deg", 180.0), "fov"),
        ("eye=target", lambda v, p: p.camera_VO.eye.__setitem__(2, 0.0), "degenerate"),
        ("up parallel", lambda v, p: p.camera_VO.up.__setitem__(1, 0.0) or p.camera_VO.up.__setitem__(2, 1.0),
         "degenerate"),
    ]
    for name, mutate, msg in cases:
        v, p = good()
        mutate(v, p)
        assert call(v, p) == V.VDI_ERR_ARG, name
        assert msg in V.last_error(), (name, V.last_error())
    v, p = good()
    v.data = None
    assert call(v, p) == V.VDI_ERR_ARG
