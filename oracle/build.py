"""Compile the plain-C oracle into ``oracle/liboracle.so`` (gcc, OpenMP, no FMA contraction), and
the same source with multiply-adds contracted into FMAs into ``oracle/liboracle_fma.so``: the
spread between the two is the oracle's own rounding noise, the envelope that long recurrences
(200 KPM steps) are judged against.

Test infrastructure: the checker the HIP library is compared with.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
LIB_FMA = os.path.join(HERE, "liboracle_fma.so")


def _compile(out: str, contract: list, verbose: bool) -> None:
    src = os.path.join(HERE, "oracle.c")
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", *contract,
           "-fno-fast-math", "-Wall", "-Wextra", "-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)


def build(verbose: bool = False) -> str:
    _compile(LIB, ["-ffp-contract=off"], verbose)
    _compile(LIB_FMA, ["-ffp-contract=fast", "-mfma"], verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
