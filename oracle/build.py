"""Compile the C oracle into oracle/liboracle.so (test infrastructure only)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
# -ffp-contract=off: no fused multiply-add, every FP32 operation rounds on its own.
# No -ffast-math and no -march=native (the library also runs on other hosts).
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-Wall", "-Wextra", "-D_GNU_SOURCE"]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, f) for f in ("mmas_oracle.c", "learned_oracle.c")]
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, "-o", tmp, *srcs, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
