"""Build the oracle's shared library (test infrastructure only).

The oracle is plain C compiled with gcc; it is never linked into, loaded by
or called from the GPU library.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB):
        return LIB
    src = os.path.join(HERE, "oracle.c")
    tmp = LIB + ".tmp"
    subprocess.check_call([
        "gcc", "-O2", "-std=gnu11", "-Wall", "-Wextra", "-ffp-contract=off", "-fopenmp",
        "-fPIC", "-shared", "-o", tmp, src, "-lm",
    ])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
