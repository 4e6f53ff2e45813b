"""MI355X (gfx950) library for ABFT-protected stencil sweeps (Cavelan & Ciorba).

The compute path is libabft_stencil.so (HIP kernels behind the C interface in
include/abft_stencil.h); ``abft`` is its Python binding.
"""
