"""MI355X (gfx950) implementation of the hot path of "Rapid Light Field Depth
Estimation with Semi-Global Matching": liblf.so (HIP kernels behind the C ABI of
include/lf.h) and its ctypes binding, `paper_1907_13449_amd.lf`."""
