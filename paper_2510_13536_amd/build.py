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
    """Compiles every source to its own object (in parallel, in a temporary
    folder), then links them into libmwcg.so."""
    import tempfile
    cc = hipcc()
    common = [f for f in flags(arch) if f != "-shared"] + list(extra or [])
    with tempfile.TemporaryDirectory(prefix="mwcg_build_") as tmpdir:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(tmpdir, os.path.splitext(src)[0] + ".o")
            cmd = [cc, *common, "-c", "-o", obj, os.path.join(CSRC, src)]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((cmd, subprocess.Popen(cmd)))
            objs.append(obj)
        failed = [cmd for cmd, pr in procs if pr.wait() != 0]
        if failed:
            raise subprocess.CalledProcessError(1, failed[0])
        tmp = LIB + ".tmp"
        cmd = [cc, "--offload-arch=" + arch, "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
