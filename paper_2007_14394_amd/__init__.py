"""MI355X (gfx950) implementation of the SDFDDGI per-frame probe update.

The work runs in ``lib/libsdfddgi.so`` (HIP kernels behind the C ABI of
``include/sdfddgi.h``); ``paper_2007_14394_amd.sdfddgi`` is its ctypes binding
with the same function names. Build with ``paper_2007_14394_amd.build.build()``.
"""
from .build import LIB_PATH  # noqa: F401
