"""The persistent served kernel's tile and counter layout, built for the
host (hipcc; nothing runs on a GPU): tiles per XCD group add up to the job's
tiles, completion counters sit on lines of their own, and a job's tiles
finishing in random order across the groups report it finished exactly once,
at its last tile."""
import ctypes
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_persistent_layout_and_completion_counting(tmp_path):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    out = str(tmp_path / "libpersist_host.so")
    cmd = ["hipcc", "--offload-arch=gfx950", "-O2", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_2206_08660_amd", "csrc"),
           os.path.join(HERE, "host", "persist_host.hip"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    L = ctypes.CDLL(out)
    L.persist_layout_check.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint]
    assert L.persist_layout_check(40000, 2000, 7) == 0
