"""Build libvdi.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(REPO, "include")
LIB = os.path.join(PKG, "libvdi.so")
SOURCES = ["vdi_api.hip", "vdi_kernels.hip", "vdi_serve.hip", "vdi_generate.hip"]
ARCH = os.environ.get("VDI_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
    # Packed FP32 instructions stay off: the compiler's scalar FP32 code is used.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I" + INCLUDE, "-I" + CSRC,
]


def build(verbose: bool = True) -> str:
    """Compile every source to an object file, then link the shared library."""
    t = time.time()
    objs = []
    os.makedirs(os.path.join(PKG, "_build"), exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(PKG, "_build", src.replace(".hip", ".o"))
        cmd = ["hipcc", *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed for " + src)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run(["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs], check=True)
    os.replace(tmp, LIB)
    if verbose:
        print(f"[build] {os.path.relpath(LIB, REPO)} ({ARCH}) in {time.time() - t:.1f}s", flush=True)
    return LIB


if __name__ == "__main__":
    build()
