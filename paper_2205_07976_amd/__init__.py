"""MI355X X-ray tracing of crystal diffraction images.

``paper_2205_07976_amd.xrt`` is the Python binding of libxrt.so (the C ABI in
include/xrt.h); ``paper_2205_07976_amd.build`` compiles it for gfx950.
"""
from . import xrt  # noqa: F401  (the library itself is loaded on first use)

__all__ = ["xrt"]
