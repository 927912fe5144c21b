"""MI355X-native (gfx950) contrastive image-encoder hot path.

The compute lives in libvl.so (HIP kernels behind the C ABI of
include/vl.h); `vl` is its ctypes binding.  Importing the package does not
load the library; the first call does, and raises if it is not built.
"""
from . import vl  # noqa: F401

__all__ = ["vl"]
