"""MI355X (gfx950) library for inner-outer Krylov recycling in diffuse optical
tomography (arXiv:1602.00138): the sequence of SPD solves that builds the global
reduced basis.

  paper_1602_00138_amd.rom     -- ctypes binding of the C ABI (include/rom.h)
  paper_1602_00138_amd.driver  -- torch-allocated buffers around the ABI calls
  paper_1602_00138_amd.build   -- hipcc build of librom.so

The binding fails to import when librom.so has not been built; there is no
fallback path.
"""
