"""Build the oracle's shared library with gcc (IEEE semantics, no FMA
contraction, OpenMP over samples): liboracle.so at -O2 for the tests, and
liboracle_fast.so at -O3 -march=native for the timed CPU baseline (the same
source and arithmetic).  Test infrastructure only."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
LIB_FAST = os.path.join(HERE, "liboracle_fast.so")
OPT = {"default": (LIB, ["-O2"]), "fast": (LIB_FAST, ["-O3", "-march=native"])}


def build(force: bool = True, variant: str = "default") -> str:
    lib, opt = OPT[variant]
    src = os.path.join(HERE, "oracle.c")
    deps = [src, os.path.join(HERE, "oracle.h")]
    if not force and os.path.exists(lib) and all(os.path.getmtime(lib) >= os.path.getmtime(d)
                                                 for d in deps):
        return lib
    cmd = ["gcc", *opt, "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-Wall", "-Wextra", "-Wno-unused-parameter",
           src, "-o", lib + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


def build_all(force: bool = True):
    return [build(force, v) for v in OPT]


if __name__ == "__main__":
    print(build_all(force="--if-stale" not in sys.argv))
