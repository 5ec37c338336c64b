"""Compile the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so
(the D3Q27 model and the D2Q9 model of App. B).

Plain gcc, OpenMP, no fused multiply-add contraction, no fast-math: the oracle
rounds every operation as written.  Built for x86-64-v3 (AVX2/FMA class hosts)
so the same shared object runs on this machine and on the GPU hosts.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "cmlbm_oracle.c"),  # D3Q27 model of Sec. II
        os.path.join(HERE, "d2q9_oracle.c"),   # D2Q9 model of App. B
        os.path.join(HERE, "mhd_oracle.c")]    # magnetic lattice of App. C and the Lorentz force
LIB = os.path.join(HERE, "liboracle.so")
LIB_EXT = os.path.join(HERE, "liboracle_ext.so")  # same source in 80-bit long double

CFLAGS = ["-O3", "-march=x86-64-v3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-shared", "-fPIC", "-Wall", "-Wextra"]


def build_one(lib, defines, force):
    if not force and os.path.exists(lib) and os.path.getmtime(lib) >= max(os.path.getmtime(s) for s in SRCS):
        return lib
    tmp = lib + ".tmp"
    subprocess.run(["gcc", *CFLAGS, *defines, "-o", tmp, *SRCS, "-lm"], check=True)
    os.replace(tmp, lib)
    return lib


def build(force=True, extended=False):
    """Build the FP64 oracle (and the 80-bit one); return the requested path."""
    a = build_one(LIB, [], force)
    b = build_one(LIB_EXT, ["-DORC_EXTENDED"], force)
    return b if extended else a


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
