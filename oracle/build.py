"""Compile the CPU oracle into oracle/liboracle.so (test infrastructure only).

Plain C99, -O2, no fast-math and no floating-point contraction, so every
float operation is the IEEE operation written in the source.  OpenMP runs the
independent per-Gaussian and per-tile loops of the splat and the per-page
k-means of the LOD levels on several threads (or_set_threads; the results do
not depend on the count).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["or_math.c", "or_create.c", "or_frame.c", "or_mlp.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    cmd = ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-fno-strict-aliasing", "-D_GNU_SOURCE", "-fopenmp", "-Wall", "-Wno-unused-function",
           "-o", LIB + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
