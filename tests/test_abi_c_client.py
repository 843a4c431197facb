"""A plain C program against include/vdi.h and libvdi.so: it compiles and
links on the host (CPU suite), and on an MI355X it renders a two-slab VDI
exactly and in preview and checks the image against the closed form."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_2206_08660_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.fixture(scope="module")
def client(tmp_path_factory):
    if shutil.which("gcc") is None or not os.path.exists(os.path.join(PKG, "libvdi.so")):
        pytest.skip("gcc or libvdi.so not available")
    exe = str(tmp_path_factory.mktemp("abiclient") / "abi_client")
    cmd = ["gcc", "-std=c11", "-O1", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROCM, "include"),
           os.path.join(HERE, "host", "abi_client.c"), "-o", exe,
           "-L" + PKG, "-lvdi", "-Wl,-rpath," + PKG, "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return exe


def test_c_client_compiles_and_links(client):
    assert os.path.exists(client)


@pytest.mark.gpu
def test_c_client_renders_the_closed_form(client):
    r = subprocess.run([client], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0 and "abi_client: ok" in r.stdout
