"""Build tests/c_abi/capi_check (a host program that calls libsat.so through include/sat.h only)
with hipcc, linked against the in-tree libsat.so.  Run after the library is built."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PKG = os.path.join(ROOT, "paper_2410_16291_amd")
SRC = os.path.join(HERE, "capi_check.cpp")
EXE = os.path.join(HERE, "capi_check")


def build(verbose: bool = False) -> str:
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    from paper_2410_16291_amd.build import hipcc   # the library's own compiler lookup
    tmp = EXE + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-O2", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include"), SRC, "-L" + PKG, "-lsat",
           "-Wl,-rpath," + PKG, "-Wl,-rpath,$ORIGIN/../../paper_2410_16291_amd", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building capi_check")
    os.replace(tmp, EXE)
    return EXE


if __name__ == "__main__":
    print(build(verbose=True))
