"""MI355X (gfx950) implementation of the massive pseudo-random number
generator of the cf4ocl paper's example application (Section 5; Listings S4
and S5): seeding and generation in hand-written HIP kernels behind a C ABI
(include/rngx.h), with a ctypes binding in :mod:`paper_1609_01257_amd.rngx`.
"""
__all__ = ["rngx", "inputs"]
