"""Multi-word-precision (DW, QDW, TW, QTW) Conjugate Gradient for MI355X.

The compute path is the HIP library `libmwcg.so` (C ABI declared in
include/mw.h); `paper_2510_13536_amd.mw` is its thin Python binding and
`paper_2510_13536_amd.problems` holds the seeded input generators.
Importing the package loads nothing: the library is opened on first use of
the binding and a missing build raises an error.
"""
__all__ = ["mw", "problems"]
