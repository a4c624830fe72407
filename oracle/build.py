"""Build the FP64 CPU oracle (test infrastructure only) into oracle/liborc.so.

Plain C99, -O2, no fast-math, no FMA contraction, OpenMP over grid points.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["eos.c", "fd.c", "c2p.c", "ccz4.c", "grmhd.c", "rhs.c"]
EXTRA = ["m1.c", "mlp.c", "amr.c", "diag.c", "les.c"]


def build(verbose=False):
    srcs = [os.path.join(HERE, s) for s in SOURCES + EXTRA if os.path.exists(os.path.join(HERE, s))]
    out = os.path.join(HERE, "liborc.so")
    cmd = ["gcc", "-std=gnu99", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wno-unused-function", "-o", out + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
