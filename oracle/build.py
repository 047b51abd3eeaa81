"""Build the FP64 CPU oracle library (test infrastructure only).

    python -m oracle.build        # writes oracle/libcholinv_oracle.so

Compiled with plain gcc, no fast-math and no floating-point contraction, so
every operation rounds as written in the C source.  OpenMP is enabled only for
the all-cores batch loop (or_inv_prop_batched_omp_*); every other routine is
single-threaded.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cholinv_oracle.c")
SRC_Q15 = os.path.join(HERE, "cholinv_oracle_q15.c")
LIB = os.path.join(HERE, "libcholinv_oracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-fopenmp", "-Wall", "-Wextra", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", *CFLAGS, "-o", tmp, SRC, SRC_Q15, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
