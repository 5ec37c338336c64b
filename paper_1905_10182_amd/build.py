"""Build the gfx950 shared libraries of the package in-tree with hipcc.

    python -m paper_1905_10182_amd.build

produces paper_1905_10182_amd/libcmlbm.so (the D3Q27 solver, C ABI in
include/cmlbm.h), libcmlbm2d.so (the D2Q9 model of App. B, C ABI in
include/cmlbm2d.h), libcmlbm_mhd.so (the magnetic lattice of App. C and the
Lorentz force, C ABI in include/cmlbm_mhd.h) and libcmnn.so (the warm-start network kernels, C ABI in
include/cmnn.h).  Cross-compiles on a machine without a GPU.
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are switched off for every HIP translation unit.
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-I" + INCLUDE, "-I" + CSRC]

LIBS = {
    "libcmlbm.so": ["cmlbm.hip"],
    "libcmlbm2d.so": ["cmlbm2d.hip"],
    "libcmlbm_mhd.so": ["cmlbm_mhd.hip"],
    "libcmnn.so": ["cmnn.hip"],
}


def build_one(name, sources, verbose=False):
    out = os.path.join(PKG, name)
    tmp = out + ".tmp"
    cmd = [HIPCC, *HIPFLAGS, *[os.path.join(CSRC, s) for s in sources], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {name}:\n{errs}")
    os.replace(tmp, out)
    return out


def build(verbose=False):
    return [build_one(n, s, verbose) for n, s in LIBS.items()]


if __name__ == "__main__":
    for p in build(verbose="-v" in sys.argv):
        print(p)
