"""Builds libmwcg.so (HIP, gfx950) in-tree with hipcc.

Flags that matter for correctness:
  -ffp-contract=off   no implicit fusion: the error-free transformations
                      rely on every +, -, * rounding once, and every
                      intended fma is written out;
  -fno-fast-math      IEEE semantics, FP64 denormals kept;
  -packed-fp32-ops off (target feature) the packed FP32 forms are not used.
"""
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libmwcg.so")
SOURCES = ["mw_blas.hip", "mw_cg.hip", "mw_batch.hip", "mw_tune.hip"]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags(arch="gfx950"):
    return ["--offload-arch=" + arch, "-O3", "-std=c++17", "-fPIC", "-shared",
            "-ffp-contract=off", "-fno-fast-math",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-I" + INCLUDE, "-I" + CSRC]


def build(verbose=False, arch="gfx950", extra=None):
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *flags(arch), *(extra or []), "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
