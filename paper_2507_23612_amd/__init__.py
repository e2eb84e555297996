"""MI355X (gfx950) library for the Chebyshev-filtered subspace iteration of
real-space Hubbard-corrected DFT (arXiv:2507.23612).

The compute path is the C-ABI library libhcu.so (include/hubbard_chfsi.h),
built from csrc/ by ``python -m paper_2507_23612_amd.build``; ``hcu`` is its
ctypes binding.  Importing this package does not load the library.
"""
__all__ = ["hcu", "build"]
