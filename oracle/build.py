"""Compile the C oracle (test infrastructure) into oracle/libsat_oracle.so with gcc.

The oracle is plain serial C; it is built with -O2 and without -ffast-math so that every
floating-point operation keeps its IEEE meaning.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sat_oracle.c")
LIB = os.path.join(HERE, "libsat_oracle.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-fno-fast-math", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
