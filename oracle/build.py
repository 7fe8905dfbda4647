"""Compile the CPU oracle (test infrastructure) into oracle/liborbf_oracle.so.

Plain C, FP64, no BLAS; -ffp-contract=off keeps every product and sum
separately rounded.  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark load the result.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "orbf_oracle.c")
LIB = os.path.join(HERE, "liborbf_oracle.so")


def build(verbose=False):
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-Wno-unused-parameter", "-o", LIB, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
