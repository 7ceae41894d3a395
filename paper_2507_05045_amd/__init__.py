"""MI355X-native exact solver for the feasibility market split problem.

The solve runs in hand-written HIP kernels behind the C ABI of ``libmsp.so``
(declared in ``include/msp.h``); ``paper_2507_05045_amd.msp`` is the thin
ctypes binding with the same names.  Importing this package does not load
the native library; ``msp`` does, and fails loudly when it is missing.
"""
