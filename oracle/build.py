"""Builds the FP64 CPU oracle (test infrastructure) with gcc, and the same
source as a float32 evaluation of its value path (used only to check the
oracle's float32 sensitivity estimates)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liborc.so")
LIB32 = os.path.join(HERE, "liborc32.so")
SRC = os.path.join(HERE, "irf_oracle.c")
FLAGS = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-Wall",
         "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    for out, extra in ((LIB, []), (LIB32, ["-DORC_REAL=float", "-fsingle-precision-constant"])):
        cmd = FLAGS + extra + ["-o", out, SRC, "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
