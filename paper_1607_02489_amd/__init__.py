"""EMIN-AMG grid-transfer setup for Q2-Q1 saddle systems on MI355X.

Submodules:
  synth  -- seeded synthetic Q2-Q1 Stokes/Oseen inputs (no method arithmetic)
  emin   -- ctypes binding of the HIP C-ABI library (libemin.so)
  build  -- builds libemin.so with hipcc for gfx950
"""
__version__ = "0.1.0"
