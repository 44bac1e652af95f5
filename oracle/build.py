"""Build step for the FP64 CPU oracle (test infrastructure only).

Compiles ``dgbgk_oracle.c`` into ``liboracle.so`` beside it with gcc, with
``-ffp-contract=off`` so every expression is evaluated as written, and OpenMP
for the element loops.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dgbgk_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [
        "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
        "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared", "-Wall",
        "-o", tmp, SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
