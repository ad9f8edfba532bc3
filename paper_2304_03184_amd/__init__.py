"""MI355X (gfx950) hot path of Instant-NVR's radiance-field back-end.

The compute lives in libnvr.so (HIP kernels behind the C ABI declared in
include/nvr.h); this package only binds it.  Importing the package does not
load the library; ``paper_2304_03184_amd._lib.lib()`` does, and raises when
the library has not been built.
"""
__all__ = ["_lib", "ops", "field", "build"]
