"""Child process of test_gpu_serve.py (run with GPU_MAX_HW_QUEUES=16 in its
environment): with a long request on a server, vdi_create of another VDI
returns while the request is still in flight, i.e. it waited only for its
own upload stream.  With the runtime's default of four hardware queues a new
stream can share a queue with a busy server stream and then waits behind its
batch; with sixteen, the server's streams and the VDI's get queues of their
own.  Prints "create: ok" on success."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import torch  # noqa: E402

import inputs  # noqa: E402
from paper_2206_08660_amd import serve  # noqa: E402
from paper_2206_08660_amd import vdi as V  # noqa: E402


def main():
    torch.cuda.set_device(0)
    tiny = inputs.load_workload("tiny", keep_dvr=False)
    w720 = inputs.load_workload("720p", keep_dvr=False)
    with V.Vdi(w720, store="f16") as h720:
        buf = torch.empty((720, 1280, 4), dtype=torch.float32, device="cuda")
        V.Vdi(tiny).close()   # first create: the library's pinned upload buffers
        torch.cuda.synchronize()
        with serve.Server(2 ** 34, max_inflight=8) as srv:
            t = srv.submit(h720, inputs.orbit_camera(40.0), 1280, 720, 1.0, 0.002, buf)   # about 70 ms
            assert t is not None
            h = V.Vdi(tiny)
            waited = srv.poll(t)
            print(f"request done when vdi_create returned: {waited}", flush=True)
            srv.drain()
            h.close()
            assert not waited, "vdi_create waited for the server's batch"
    print("create: ok", flush=True)


if __name__ == "__main__":
    main()
