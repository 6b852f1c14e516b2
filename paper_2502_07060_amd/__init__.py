"""MI355X-native batched Berends-Giele recursion for n-gluon tree amplitudes.

Public modules
--------------
bg      ctypes binding of the C-ABI library ``libbg_mi355x.so``: the entry
        points ``bg_amplitudes_c128`` and ``bg_amplitudes_fp`` (and the rest
        declared in ``include/bg.h``) under the same names.  Loading it does not
        touch the GPU; calling a compute entry point needs one.
inputs  seeded synthetic phase-space points and polarisation vectors
        (numpy, host side); no recursion arithmetic lives there.

Importing the package loads nothing native; ``paper_2502_07060_amd.bg`` loads
the shared library on first use and raises if it has not been built.
"""
__all__ = ["bg", "inputs"]
