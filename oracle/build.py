"""Build the oracle's C part (test infrastructure only).

Compiles ``oracle/fdtd.c`` into ``oracle/liborc_fdtd.so`` with gcc, plain
``-O2`` (no fast-math, no FMA contraction) and OpenMP over z-planes.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fdtd.c")
LIB = os.path.join(HERE, "liborc_fdtd.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
           "-shared", "-std=c11", "-D_GNU_SOURCE", SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
