"""Build the oracle's C eigensolver (test infrastructure only).

``python -m oracle.build`` or ``oracle.build.build()`` compiles ``jacobi.c``
with gcc into ``liboracle_jacobi.so`` beside it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "jacobi.c")
LIB = os.path.join(HERE, "liboracle_jacobi.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99", SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
