"""Build the oracle's C library (``oracle/liboracle.so``) with gcc.

Test infrastructure only: the oracle is the independent CPU check of the GPU
path and is never linked into it.  The flags keep IEEE double semantics: no
fast-math and no floating-point contraction (the Kahan compensation and the
4-multiply/2-add complex product must not be fused).  No ``-march=native``:
the library is built here and may run on a different host CPU.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ryser.c")
LIB = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile ryser.c into liboracle.so; return the library path."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", *CFLAGS, SRC, "-o", tmp], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
