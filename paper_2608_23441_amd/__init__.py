"""MI355X (gfx950) circulant inverse PFB and up-channelization.

The computation lives in libipfb.so (HIP kernels behind a C ABI, declared in
include/ipfb.h); `ipfb` is its thin Python binding.
"""
from . import inputs  # noqa: F401
from . import ipfb  # noqa: F401

__all__ = ["inputs", "ipfb"]
