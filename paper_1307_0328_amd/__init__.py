"""MI355X (gfx950) implementation of the data-parallel sweep of the
parallelized multiple-worm algorithm (PMWA, arXiv:1307.0328).

The compute path is libpmwa.so (HIP kernels behind a C ABI, include/pmwa.h);
``paper_1307_0328_amd.pmwa`` is its ctypes binding.
"""
