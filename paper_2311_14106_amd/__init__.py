"""MI355X-native hot path of mode-optimized ab initio DMRG (arXiv:2311.14106).

The computation lives in libmdmrg.so (C++ host engine + HIP kernels for
gfx950) behind the C ABI of include/mdmrg.h; ``mdmrg`` is its thin ctypes
binding.  Importing this package does not load the library; the binding
loads it on first use and raises if it has not been built.
"""
__all__ = ['mdmrg', 'build']
