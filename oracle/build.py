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


def build_sanitized(out: str) -> str:
    """The same source with AddressSanitizer and UndefinedBehaviorSanitizer
    (every undefined-behaviour report fatal), for a checking run of the
    oracle's C routines: a Python process loads it with the sanitizer
    runtimes preloaded and RP_ORACLE_LIB naming it."""
    src = os.path.join(_HERE, "oracle.c")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-fPIC", "-shared",
           "-fno-fast-math", "-ffp-contract=off", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
           src, "-o", out, "-lm"]
    subprocess.check_call(cmd)
    return out


def sanitizer_preload() -> str:
    """LD_PRELOAD value for a process that loads the sanitized build."""
    libs = []
    for name in ("libasan.so", "libubsan.so"):
        libs.append(subprocess.check_output(["gcc", f"-print-file-name={name}"], text=True).strip())
    return " ".join(libs)


if __name__ == "__main__":
    print(build())
