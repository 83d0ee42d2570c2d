"""Builds the C oracle into oracle/_lib/liboracle.so with gcc.

Test infrastructure only (see oracle/__init__.py).  IEEE binary64 with
floating-point contraction switched off, so every product and sum rounds as
written; OpenMP parallelises the per-node loops, which are independent.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "_lib", "liboracle.so")


def compile_source(src, out, verbose=False, quiet=False):
    """Compiles one C source into a shared library with the oracle's flags
    (quiet: compiler messages are not shown)."""
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-fopenmp", "-Wall", "-Wextra", "-o", out, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True, capture_output=quiet)
    return out


def build(verbose=False):
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    compile_source(SRC, tmp, verbose)
    os.replace(tmp, LIB)
    return LIB


def ensure_built():
    """Builds the oracle when no built library is present or the source is
    newer than it."""
    if not os.path.exists(LIB) or os.path.getmtime(SRC) > os.path.getmtime(LIB):
        build()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
