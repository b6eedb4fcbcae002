"""Builds the CPU oracle (test infrastructure): oracle/libmwo.so and the
op-counting variant oracle/libmwo_count.so.

The oracle is compiled with contraction off so that every fused
multiply-add is an explicit fma() and every other operation rounds once.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mwo.c")
FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11", "-shared", "-fPIC", "-Wall", "-Wno-unknown-pragmas"]


def build(verbose=False):
    outs = []
    for name, extra in (("libmwo.so", ["-fopenmp"]), ("libmwo_count.so", ["-DMWO_COUNT_OPS"])):
        out = os.path.join(HERE, name)
        cmd = ["gcc", *FLAGS, *extra, "-o", out + ".tmp", SRC, "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
        outs.append(out)
    return outs


if __name__ == "__main__":
    for p in build(verbose="-v" in sys.argv):
        print(p)
