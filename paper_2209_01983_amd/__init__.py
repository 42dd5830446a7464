"""MI355X-native SALE Lagrange + Eulerian-remap step (ScalSALE, arXiv 2209.01983).

The step runs in hand-written HIP kernels for gfx950 behind the C-ABI library
``libsale.so`` (declared in ``include/sale.h``); ``sale`` is its thin ctypes
binding. Importing this package loads nothing; the library is loaded on the
first call and a missing build raises an error.
"""
