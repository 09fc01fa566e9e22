"""Block incomplete LU (BILU, arXiv 1908.10169) on AMD Instinct MI355X.

The compute path is libbilu.so (HIP kernels for gfx950 + host C++ behind the
C ABI in include/bilu.h); ``bilu`` is its thin Python binding and
``matgen`` the seeded synthetic workloads.  Nothing is loaded at import.
"""
