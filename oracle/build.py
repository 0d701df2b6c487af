"""Build the CPU FP64 oracle library (``liboracle.so``) from ``spgm_oracle.c``.

Test infrastructure only: the oracle is compiled with gcc, OpenMP and no fast-math,
and is never linked into the product library.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "spgm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build_oracle(verbose: bool = False) -> str:
    """Compile ``liboracle.so`` in place and return its path (always recompiles)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-fno-fast-math", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def ensure_oracle() -> str:
    """Return the library path, building it only when it is missing or stale."""
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        return build_oracle()
    return LIB


if __name__ == "__main__":
    print(build_oracle(verbose=True))
