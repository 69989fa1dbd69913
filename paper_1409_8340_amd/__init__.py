"""MI355X-native implicit TDGL solver (Sadovskyy et al., arXiv:1409.8340).

The solver itself is the C-ABI library ``libtdgl.so`` (HIP kernels for
gfx950); ``paper_1409_8340_amd.tdgl`` is its thin ctypes binding.  Importing
this package does not load the library; creating a solver does, and fails
loudly when the library has not been built.
"""
