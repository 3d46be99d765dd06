"""Pre-packed tall-and-skinny matrix multiply (AutoTSMM) for MI355X / gfx950.

The compute path is ``libtsmm.so`` (hand-written HIP kernels behind a C ABI,
declared in ``include/tsmm.h``); :mod:`paper_2208_08088_amd.tsmm` is the thin
Python binding with the same names.  Nothing is imported here, so the input
generators (:mod:`paper_2208_08088_amd.inputs`) stay usable on hosts where
the library has not been built.
"""
