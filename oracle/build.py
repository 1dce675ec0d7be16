"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc -O3, OpenMP, no floating-point contraction and no reassociation, so
every product and sum is rounded exactly as written (vectorisation does not
change a result).  ISA level x86-64-v3 (AVX2), which every host this runs on
has, rather than -march=native, so the library built here also loads there.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["bd3mg_oracle.c", "convnet_oracle.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wno-unknown-pragmas",
           "-o", LIB + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
