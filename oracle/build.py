"""Compile the C oracle into oracle/liboracle.so (test infrastructure only).

build(native=True) writes oracle/liboracle_native.so instead, compiled for the
host CPU it runs on (-march=native): the benchmark's CPU baseline times that
build. Contraction stays off, so both builds round every FP32 operation the
same way and give the same results."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
# -ffp-contract=off: no fused multiply-add, every FP32 operation rounds on its own.
# No -ffast-math; -march=native only in the separate native build.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-Wall", "-Wextra", "-D_GNU_SOURCE"]


NATIVE_LIB = os.path.join(HERE, "liboracle_native.so")


def build(verbose: bool = False, native: bool = False) -> str:
    srcs = [os.path.join(HERE, f) for f in ("mmas_oracle.c", "learned_oracle.c")]
    out = NATIVE_LIB if native else LIB
    tmp = out + f".tmp{os.getpid()}"
    cmd = ["gcc", *CFLAGS, *(["-march=native"] if native else []), "-o", tmp, *srcs, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
