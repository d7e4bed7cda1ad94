"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

The C oracle (oracle/sat_oracle.c) and the library's host code (argument validation, planning and
launch preparation in csrc/sat_api.cpp and the launchers; device code is compiled as usual) are
built with -fsanitize=address,undefined, and the CPU tests that drive them -- the C ABI's
validation of every call, and the oracle against its pins, streamed and in bands -- run again in a
child process against those builds, with the sanitizer runtime preloaded.  Any heap or stack
overflow, use after free or undefined behaviour fails the run.  A planted overflow checks first
that the runtime is active in that setup.

The sanitized builds go to _build/sanitize/ and are reused while their sources are unchanged.
"""
import hashlib
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "sanitize")
CSRC = os.path.join(ROOT, "paper_2410_16291_amd", "csrc")
LIB_SOURCES = ["sat_api.cpp", "sat_build.hip", "sat_gather.hip", "sat_upload.hip"]
CLANG = "/opt/rocm/llvm/bin/clang"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-shared-libsan", "-fno-omit-frame-pointer"]
CHILD_TESTS = ["tests/test_abi.py", "tests/test_oracle.py", "tests/test_oracle_stream.py", "tests/test_oracle_bands.py",
               "tests/test_oracle_moments.py", "tests/test_banded_compare.py"]


def runtime():
    libs = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return libs[-1] if libs else None


def digest(paths, extra):
    h = hashlib.sha256(" ".join(extra).encode())
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def build_if_stale(out, sources, cmd):
    stamp = out + ".src"
    key = digest(sources, cmd)
    if os.path.exists(out) and os.path.exists(stamp) and open(stamp).read() == key:
        return out
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    with open(stamp, "w") as f:
        f.write(key)
    return out


@pytest.fixture(scope="module")
def builds():
    if runtime() is None or not os.path.exists(CLANG):
        pytest.skip("the ROCm clang sanitizer runtime is not installed")
    from paper_2410_16291_amd import build as lib_build
    os.makedirs(OUT, exist_ok=True)
    oracle_src = os.path.join(ROOT, "oracle", "sat_oracle.c")
    oracle_lib = os.path.join(OUT, "libsat_oracle_san.so")
    build_if_stale(oracle_lib, [oracle_src],
                   [CLANG, "-O1", "-g", "-std=c11", "-fPIC", "-shared"] + SAN + ["-o", oracle_lib, oracle_src, "-lm"])
    srcs = [os.path.join(CSRC, s) for s in LIB_SOURCES] + glob.glob(os.path.join(CSRC, "*.h")) + \
        [os.path.join(ROOT, "include", "sat.h")]
    lib = os.path.join(OUT, "libsat_san.so")
    host_san = []
    for f in SAN:                       # sanitizers on the host pass only, never in device code
        host_san += ["-Xarch_host", f]
    cmd = ([lib_build.hipcc(), "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=off", "-Wno-unused-function",
            "-I" + os.path.join(ROOT, "include"), "-I" + CSRC] + host_san +
           ["-o", lib] + [os.path.join(CSRC, s) for s in LIB_SOURCES])
    build_if_stale(lib, srcs, cmd)
    return lib, oracle_lib


def child_env(lib, oracle_lib):
    env = dict(os.environ)
    env.update({"SAT_LIBRARY": lib, "SAT_ORACLE_LIBRARY": oracle_lib, "LD_PRELOAD": runtime(),
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=86",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=87"})
    return env


def test_planted_overflow_is_caught(builds, tmp_path):
    """The sanitizer runtime is live in a Python child process that loads a sanitized library."""
    src = tmp_path / "planted.c"
    src.write_text("#include <stdlib.h>\nint planted(int i) { char *p = malloc(8); int v = p[i]; free(p); "
                   "return v; }\n")
    so = tmp_path / "planted.so"
    subprocess.run([CLANG, "-O0", "-g", "-fPIC", "-shared"] + SAN + ["-o", str(so), str(src)], check=True)
    code = "import ctypes; ctypes.CDLL(%r).planted(16)" % str(so)
    r = subprocess.run([sys.executable, "-c", code], env=child_env(*builds), capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr, r.stderr[-2000:]


def test_cpu_suite_under_sanitizers(builds):
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"] +
                       CHILD_TESTS, cwd=ROOT, env=child_env(*builds), capture_output=True, text=True, timeout=1200)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
