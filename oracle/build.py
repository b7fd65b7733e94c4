"""Build the FP64 CPU oracle (test infrastructure) into oracle/libora.so with gcc.

The oracle is compiled without fast-math and without floating-point contraction so that
its results follow the C source operation by operation.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libora.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
        "-std=c11", "-Wall", "-Wextra", "-o", LIB + ".tmp", os.path.join(HERE, "ora.c"), "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
