"""MI355X (gfx950) Darknet-style CNN forward library.

``libdn.so`` (built from ``csrc/`` by ``build.py``) holds the HIP kernels and
the C ABI declared in ``include/dn.h``; ``dn.py`` is its ctypes binding and
``serve.py`` the continuous-batching serving loop on top of it.  Importing
``paper_1811_03882_amd.dn`` fails if the library has not been built.
"""
