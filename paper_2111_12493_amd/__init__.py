"""MI355X-native hash-based k-bisimulation (graph summarization).

The compute path is a C-ABI shared library of hand-written HIP kernels for
gfx950 (``csrc/``, declared in ``include/bsim.h``); ``binding`` is a thin
ctypes layer over it.  ``graphgen`` produces seeded synthetic input graphs.
Importing this package loads nothing; the binding loads the library on first
use and raises if it has not been built.
"""
