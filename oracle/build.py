"""Compile the CPU oracle into ``oracle/liblbgk_oracle.so`` with gcc.

Test infrastructure: the oracle is the FP64 reference the GPU library is
checked against; it is never part of the product path.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbgk_oracle.c")
LIB = os.path.join(HERE, "liblbgk_oracle.so")


FLAGS = ["-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
         "-fopenmp", "-Wall"]


def build(verbose=False, src=SRC, out=LIB, extra=()):
    """Compile `src` (the oracle source, or a copy of it) into `out`."""
    cmd = ["gcc", *FLAGS, *extra, "-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
