"""MI355X-native (gfx950, HIP) SSP-RK3 stage of 3D ideal special-relativistic
MHD after the ECHO scheme of arXiv 2401.03008.

- ``binding``: ctypes binding of libsrmhd.so (the C ABI, include/srmhd.h)
- ``solver``: torch-owned device buffers around the ABI
- ``inputs``: seeded synthetic initial data (CPA wave, Alfvenic turbulence)
- ``build``: in-tree hipcc build of libsrmhd.so
"""
from . import inputs  # noqa: F401

__all__ = ["inputs", "binding", "solver", "build"]
