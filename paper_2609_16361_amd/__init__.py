"""MI355X-native five-field gradient-reconstruction lattice Boltzmann solver.

Submodules:
  inputs   -- seeded synthetic workloads (initial fields and lattice parameters)
  binding  -- ctypes binding of the HIP library (libgrlbm.so), same names as the C ABI
  build    -- compiles the HIP library for gfx950

Nothing is loaded at import time; `binding` loads the compiled library on first use
and raises if it is missing.
"""
