"""MI355X-native matrix-free frequency-domain FIT (hot path: operator + Krylov).

Submodules:
  fit      ctypes binding of libfit.so (the C ABI in include/fit.h)
  devices  seeded synthetic device descriptions (inputs only)
  build    hipcc build of libfit.so for gfx950
"""
__all__ = ["fit", "devices", "build"]
