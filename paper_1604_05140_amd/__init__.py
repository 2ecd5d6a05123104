"""libsgl: fast spherical Gauss-Laguerre transforms on AMD MI355X (gfx950).

The transform runs in the C-ABI library libsgl.so (HIP kernels); the Python
module `sgl` marshals arguments into it.  Nothing here computes the transform.
"""
