"""Build the CPU oracle library (test infrastructure): plain C, FP64, OpenMP.

-ffp-contract=off keeps every multiply and add separately rounded; fma() appears only
where the source writes it.  -fcx-limited-range: complex products and quotients (plain.c)
by their textbook formulas, without the inf/NaN recovery of C99 Annex G.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libnbo.so")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, "nbo.c"), os.path.join(HERE, "plain.c")]
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-fcx-limited-range", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", LIB + ".tmp", *srcs, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
