"""Build the CPU oracle (test infrastructure) as oracle/liboracle.so.

Plain C11 with gcc: -O2 and -ffp-contract=off so that every floating-point
product and sum is rounded on its own (no fused multiply-add), no fast-math,
denormals kept.  OpenMP only parallelises the synapse-sampling loop, whose
outputs have fixed positions, so the network does not depend on the thread
count.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["model.c", "network.c", "sim.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-o", tmp] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
