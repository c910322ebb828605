"""libfcirc: FFT-free f-circulant matrix-vector products on AMD MI355X (gfx950).

The HIP library (libfcirc.so, C-ABI in include/fcirc.h) does all the work; this
package holds its Python binding (``fcirc``), the build script (``build``) and the
seeded input generators (``workloads``). Importing the package does not load the
library; the first call does, and fails loudly if it has not been built.
"""
