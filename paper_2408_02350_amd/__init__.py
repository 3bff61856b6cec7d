"""MI355X-native meshfree ALE time step for the BGK equation.

Modules:
  bgk     -- Python binding of libbgk.so (the HIP kernels behind include/bgk.h)
  inputs  -- seeded cavity clouds and run parameters
  build   -- builds libbgk.so with hipcc for gfx950

Importing the package loads nothing; the library is loaded on first use.
"""
__all__ = ["bgk", "inputs", "build"]
