"""MI355X-native MPS sampling sweep (FastMPS hot path) behind a C ABI.

* ``csrc/``   HIP kernels for gfx950 and the C-ABI host code (libmps.so)
* ``mps``     ctypes binding with the C entry-point names, plus ``Sampler``
* ``synth``   seeded synthetic right-canonical MPS inputs
* ``build``   in-tree build of libmps.so
"""
