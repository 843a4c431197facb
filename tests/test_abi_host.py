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


def test_replace_rejects_null_arguments_before_any_device_work():
    lib = V.lib()
    d = V.Desc()
    assert lib.vdi_replace_begin(None, ctypes.byref(d), None) == V.VDI_ERR_ARG
    assert lib.vdi_replace_begin(ctypes.c_void_p(1), None, None) == V.VDI_ERR_ARG
    sw = ctypes.c_int32(7)
    assert lib.vdi_replace_poll(None, ctypes.byref(sw)) == V.VDI_ERR_ARG
    assert lib.vdi_replace_poll(ctypes.c_void_p(1), None) == V.VDI_ERR_ARG
