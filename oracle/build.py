"""Compiles oracle.c into liboracle.so with gcc (FP64, OpenMP, no fast-math).

Test infrastructure: the checker is built alongside the product so the tests
and the CPU baseline can load it.
"""

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def library_path() -> str:
    return os.path.join(_HERE, "liboracle.so")


def build() -> str:
    src = os.path.join(_HERE, "oracle.c")
    out = library_path()
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared",
           "-fno-fast-math", "-ffp-contract=off", "-Wall", "-Wextra",
           "-Wno-unused-parameter", src, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
