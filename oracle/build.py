"""Build the C part of the oracle (TEST INFRASTRUCTURE ONLY).

Compiles ``oracle/ndft.c`` into ``oracle/libndft.so`` with gcc and OpenMP.  The
GPU library never links this object.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ndft.c")
LIB = os.path.join(HERE, "libndft.so")


def build(force: bool = False) -> str:
    """Compile the oracle shared library; returns its path."""
    if (not force and os.path.exists(LIB)
            and os.path.getmtime(LIB) >= os.path.getmtime(SRC)):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
           "-fno-fast-math", "-ffp-contract=off", SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True))
