"""Build the oracle's shared library with gcc (plain C, -O2, no fast-math).

Test infrastructure only: the oracle checks the GPU library and is never part
of its compute path.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["dgo_basis.c", "dgo_euler.c", "dgo_mesh.c", "dgo_scheme.c", "dgo_amr.c", "dgo_api.c"]
LIB = os.path.join(HERE, "libdgo.so")


def build(verbose=False):
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-Wno-unused-function", "-o", tmp] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
