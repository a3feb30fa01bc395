"""SUPA shower propagation on MI355X (gfx950).

Submodules:
  supa       -- ctypes binding of libsupa.so (the HIP kernels behind include/supa.h)
  workloads  -- seeded synthetic initial conditions and process parameters
  build      -- in-tree build of libsupa.so with hipcc
"""
__all__ = ["supa", "workloads", "build"]
