"""Compile the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, OpenMP, no fused multiply-add contraction, no fast-math: the oracle
rounds every operation as written.  Built for x86-64-v3 (AVX2/FMA class hosts)
so the same shared object runs on this machine and on the GPU hosts.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cmlbm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O3", "-march=x86-64-v3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-shared", "-fPIC", "-Wall", "-Wextra"]


def build(force=True):
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
