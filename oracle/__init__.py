"""CPU oracle for multi-word (DW, QDW, TW, QTW) and FP64 Conjugate Gradient.

TEST INFRASTRUCTURE ONLY: this package is the plain reference the HIP path is
checked against.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import it; the product path never does.
"""
from .mwo import *  # noqa: F401,F403
