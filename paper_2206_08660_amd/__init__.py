"""MI355X-native raycasting of Volumetric Depth Images (Gupta et al., arXiv 2206.08660).

The product is libvdi.so (HIP kernels for gfx950 behind the C ABI of
include/vdi.h); `vdi` is its Python binding.
"""
from . import vdi  # noqa: F401
from .vdi import Vdi, VdiError, lowres_size  # noqa: F401
