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


VARIANTS = ((LIB, []), (LIB32, ["-DORC_REAL=float", "-fsingle-precision-constant"]))


def source_hash(extra) -> str:
    """sha256 over the oracle's sources and the compiler command of one
    build; written beside each library and compared by the loader."""
    import hashlib
    h = hashlib.sha256(" ".join(FLAGS + list(extra)).encode())
    for name in ("irf_oracle.c", "irf_oracle.h"):
        with open(os.path.join(HERE, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()


def stamp_ok(out: str) -> bool:
    extra = dict(VARIANTS)[out]
    try:
        with open(out + ".sha256") as f:
            return f.read().strip() == source_hash(extra)
    except OSError:
        return False


def build(verbose: bool = False) -> str:
    for out, extra in VARIANTS:
        cmd = FLAGS + extra + ["-o", out, SRC, "-lm"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        with open(out + ".sha256", "w") as f:
            f.write(source_hash(extra) + "\n")
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
