"""Build the oracle's C library (TEST INFRASTRUCTURE ONLY).

Compiles ``gemm_f64.c`` with the host C compiler into ``liboracle.so`` next
to this file.  The oracle is built by the same top-level build step as the
GPU library, but from its own sources and with a different compiler, so the
two share no object code.

``-ffp-contract=off`` keeps every multiply and add a separately rounded IEEE
double operation, so the summation is exactly the one the source spells out.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gemm_f64.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cc = os.environ.get("CC", "gcc")
    # a per-process name: concurrent builds (parallel test workers) each
    # write their own file and the last rename wins
    tmp = "%s.%d.tmp" % (LIB, os.getpid())
    cmd = [cc, "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-std=c11", SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
