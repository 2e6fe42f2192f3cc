"""Build the CPU oracle shared libraries (test infrastructure only).

    python oracle/build.py

Compiles abd_oracle.cpp with g++ at -O2 and -ffp-contract=off, so no
multiply-add is fused and the arithmetic is what the source says:
liboracle.so single-threaded, and liboracle_omp.so with OpenMP over
vertices, bodies and candidate pairs (every parallel loop either writes
per-element results that are then combined in list order, or takes a
minimum or a count, so both libraries compute bit-identical results).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")
LIB_SAN = os.path.join(HERE, "liboracle_san.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "abd_oracle.cpp")
    for out, extra in ((LIB, ["-Wno-unknown-pragmas"]), (LIB_OMP, ["-fopenmp"])):
        cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off",
               "-fno-fast-math", "-fPIC", "-shared", "-Wall",
               "-Wno-unused-function", *extra, src, "-o", out + ".tmp"]
        if verbose:
            print(" ".join(cmd))
        subprocess.check_call(cmd)
        os.replace(out + ".tmp", out)
    return LIB


def build_sanitized(verbose: bool = False) -> str:
    """liboracle_san.so: the single-threaded oracle with AddressSanitizer
    and UndefinedBehaviorSanitizer (any undefined-behaviour report aborts);
    load it with the sanitizer runtime preloaded (LD_PRELOAD of libasan)
    and ORACLE_LIB pointing at it."""
    src = os.path.join(HERE, "abd_oracle.cpp")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-ffp-contract=off",
           "-fno-fast-math", "-fPIC", "-shared", "-Wall",
           "-Wno-unused-function", "-Wno-unknown-pragmas",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", src, "-o", LIB_SAN + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB_SAN + ".tmp", LIB_SAN)
    return LIB_SAN


if __name__ == "__main__":
    build(verbose=True)
    if "--sanitize" in sys.argv:
        build_sanitized(verbose=True)
    sys.exit(0)
