"""MI355X-native Bicoptor 2.0 DReLU/ReLU hot path.

The compute path is libbicop.so (HIP kernels for gfx950 behind the C ABI of
include/bicop.h); ``bicop`` is its ctypes binding.  Importing ``bicop`` fails
if the library has not been built (python -m paper_2309_04909_amd.build).
"""
