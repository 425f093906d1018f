"""Build the plain multi-threaded CPU NFFT (baseline/libcpu_nfft.so) with g++ and OpenMP."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpu_nfft.cpp")
LIB = os.path.join(HERE, "libcpu_nfft.so")


def build(force: bool = False) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["g++", "-O3", "-march=x86-64-v2", "-std=c++17", "-fopenmp", "-fPIC",
                           "-shared", SRC, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True))
