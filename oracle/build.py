"""Build the FP64 CPU oracle (test infrastructure) with gcc.

The oracle is a plain C11 + OpenMP shared library, ``oracle/liblbm_oracle.so``.
It is compiled for a generic x86-64-v3 host so that the same build runs on
any recent server CPU.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liblbm_oracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "lbm_oracle.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
