"""Build the oracle's shared library (test infrastructure only).

gcc, C11, OpenMP, IEEE double with no contraction into FMAs, no
target-specific instruction sets (the library is built here and also run on
other hosts).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=gnu11", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas",
           os.path.join(HERE, "lbm_oracle.c"), "-o", LIB, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
