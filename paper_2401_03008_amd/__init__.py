"""MI355X-native (gfx950, HIP) SSP Runge-Kutta stage of 3D ideal
special-relativistic MHD after the ECHO scheme of arXiv 2401.03008.

- ``binding``: ctypes binding of libsrmhd.so (the C ABI, include/srmhd.h)
- ``solver``: torch-owned device buffers around the ABI
- ``inputs``: seeded synthetic initial data (CPA wave, 3D and 2D Alfvenic
  turbulence)
- ``learned``: the learned Newton guess (training on the library's kernels)
- ``runs``: long turbulence runs with spectra and div B logs
- ``build``: in-tree hipcc build of libsrmhd.so
"""
from . import inputs  # noqa: F401

__all__ = ["inputs", "binding", "solver", "learned", "runs", "build"]
