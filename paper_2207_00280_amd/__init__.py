"""MI355X (gfx950) B-spline element integration for IGA-FEM.

The integration itself lives in the HIP library ``libigafem.so`` (C ABI in
``include/igafem.h``); ``paper_2207_00280_amd.igafem`` is its ctypes binding.
"""
