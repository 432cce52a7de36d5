"""MI355X (gfx950) HISQ staggered Dslash and CG solvers.

The compute path is ``libhisq.so`` (hand-written HIP kernels behind the C ABI
of ``include/hisq.h``); :mod:`paper_2306_01098_amd.hisq` is its ctypes
binding and :mod:`paper_2306_01098_amd.build` compiles it for gfx950.
"""
