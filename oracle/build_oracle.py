"""Compile the CPU oracle (test infrastructure) into oracle/libteno_oracle.so with gcc.

Plain double precision, no contraction of multiply-add pairs and no fast-math, so that the
evaluation order is the one written in the source.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libteno_oracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "teno_oracle.c")
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function", "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=HERE)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
