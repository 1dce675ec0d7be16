"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, OpenMP, no floating-point contraction so every product and sum is
rounded exactly as written.  Portable ISA level so the library built here also
loads on other x86-64 hosts.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["bd3mg_oracle.c", "convnet_oracle.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    cmd = ["gcc", "-O2", "-march=x86-64-v2", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wno-unknown-pragmas",
           "-o", LIB + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
