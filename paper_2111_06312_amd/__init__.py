"""MI355X (gfx950) implicit randomized truncated SVD.

The product is libisvd.so (HIP kernels behind the C ABI of include/isvd.h);
`isvd` is its ctypes binding.
"""
