"""MI355X-native explicit material point method (MPM) step.

Submodules:
  scenes -- seeded synthetic scene inputs (no MPM arithmetic)
  mpmx   -- ctypes binding of the HIP library ``libmpmx.so`` (C ABI in
            include/mpmx.h); importing it loads the library and fails loudly
            if it has not been built.
"""
__all__ = ["scenes"]
