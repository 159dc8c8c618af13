"""MI355X (gfx950) Gauss--Newton--Krylov diffeomorphic registration engine.

The compute path is the HIP library ``libclaire_gfx950.so`` (C ABI in
include/claire.h); ``paper_2401_17493_amd.claire`` is its torch binding.
"""
