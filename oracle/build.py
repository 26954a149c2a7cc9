"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain C, gcc, -O2 with floating-point contraction off so that every product
and sum is rounded exactly where the source writes it.

`python oracle/build.py --sanitize` builds a copy instrumented with
AddressSanitizer and UndefinedBehaviorSanitizer (oracle/liboracle_san.so) and
runs the CPU test suite (-m "not gpu") against it; see sanitize().
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["oracle_math.c", "oracle_sim.c", "oracle_adjoint.c"]
LIB = os.path.join(HERE, "liboracle.so")
SAN_LIB = os.path.join(HERE, "liboracle_san.so")
SAN_FLAGS = ("-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g")


def build(verbose=False, extra_flags=(), out=LIB):
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-Wno-unused-parameter", *extra_flags, "-o", out]
    cmd += [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return out


def sanitize(pytest_args=()):
    """Build the sanitized oracle and run the CPU suite with it loaded (the
    sanitizer runtime preloaded into the Python process; leak reports off,
    since the interpreter itself keeps memory until exit).  Returns pytest's
    exit status."""
    build(verbose=True, extra_flags=SAN_FLAGS, out=SAN_LIB)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], check=True, capture_output=True,
                          text=True).stdout.strip()
    env = dict(os.environ, UGKWP_ORACLE_LIB=SAN_LIB, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    root = os.path.dirname(HERE)
    cmd = [sys.executable, "-m", "pytest", os.path.join(root, "tests"), "-q", "-m", "not gpu", *pytest_args]
    print(" ".join(cmd), flush=True)
    return subprocess.run(cmd, env=env, cwd=root).returncode


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        sys.exit(sanitize([a for a in sys.argv[1:] if a != "--sanitize"]))
    build(verbose=True, extra_flags=sys.argv[1:])
