"""MI355X-native unsplit ideal-MHD update (per-patch-group VL/CTU + CT).

Submodules:
  build   -- compiles libmhd.so (HIP, gfx950) in place
  mhd     -- ctypes binding of the C ABI declared in include/mhd.h (needs torch)
  inputs  -- seeded synthetic problems (no update arithmetic)
"""
__all__ = ["build", "inputs"]
