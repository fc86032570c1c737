"""Octree colour-quantisation background modelling on MI355X (gfx950).

The GPU library is libobg.so (HIP kernels behind a C ABI, see include/obg.h);
`paper_1412_1945_amd.obg` is its ctypes binding.
"""
