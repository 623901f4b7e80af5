"""MI355X (gfx950) approximate inverse of discrete Fourier integral operators.

The library (libfio.so, C ABI in include/fio.h) builds the butterfly factors of
K, the hierarchical inverse factors of Kd^* Kd, and applies them in HIP kernels.
This package is the thin Python binding; see ``paper_2105_02995_amd.fio``.
"""
