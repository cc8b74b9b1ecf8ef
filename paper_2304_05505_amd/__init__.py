"""THC-oo-K k-point exact exchange on gfx950 (HIP kernels behind a C ABI).

``paper_2304_05505_amd.exx`` is the ctypes binding of ``libexx.so``; import it
explicitly (it loads the library and raises if it has not been built).
``paper_2304_05505_amd.build`` compiles the library in-tree.
"""
