"""Compile the multi-core CPU baseline (sat_omp.c) into cpu_baseline/libsat_omp.so with gcc and
OpenMP.  The hot loops carry AVX2 and generic clones, picked at load time for the host CPU."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sat_omp.c")
LIB = os.path.join(HERE, "libsat_omp.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra", "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
