"""Precision studies of the solver on one GPU.

    python -m paper_1905_10182_amd.studies precision [--n 512] [--steps 2000] [--every 100]
    python -m paper_1905_10182_amd.studies kolmogorov [--n 384] [--steps 5000] [--every 500]

``precision``: the 3D Taylor-Green vortex (u0 = 0.05, Re = 1600) advanced in
lockstep with FP64, FP32, FP16 and BF16 population storage (16-bit both with
round-to-nearest and with stochastic rounding), all resident on the GPU at
once.  At every checkpoint it reports the FP64-reduced kinetic energy of each
run and the relative L2 velocity error of each run against the FP64 and the
FP32 runs.

``kolmogorov``: Kolmogorov flow (F_x = F0 sin(2 pi 4 y / N), tau = 0.5005)
with FP64, FP32 and FP16 (both roundings) storage, same report.

Both print one JSON object per checkpoint.  Error norms are taken with torch
on device-resident moments (diagnostics only; the solver runs in libcmlbm).
"""
import argparse
import json
import sys
import time

import workloads
from paper_1905_10182_amd.cmlbm import RED, Lattice


def _rel(a, b, torch):
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def lockstep(lattices, steps, every, label, out=sys.stdout):
    import torch

    names = list(lattices)
    t = 0
    rows = []
    while t <= steps:
        u = {k: lattices[k].moments()[1] for k in names}
        red = {k: lattices[k].reduce(allow_unstable=True)[0] for k in names}
        row = {"study": label, "step": t}
        for k in names:
            row[f"ke_{k}"] = float(red[k][RED["ke"]])
            row[f"umax_{k}"] = float(red[k][RED["umax"]])
            if k != "fp64" and "fp64" in u:
                row[f"err_{k}_vs_fp64"] = _rel(u[k], u["fp64"], torch)
            if k not in ("fp64", "fp32") and "fp32" in u:
                row[f"err_{k}_vs_fp32"] = _rel(u[k], u["fp32"], torch)
        del u
        print(json.dumps(row), file=out, flush=True)
        rows.append(row)
        if t == steps:
            break
        n = min(every, steps - t)
        t0 = time.perf_counter()
        for k in names:
            lattices[k].step(n)
        torch.cuda.synchronize()
        t += n
        print(f"[{label}] step {t} ({time.perf_counter() - t0:.2f} s for {n} steps x {len(names)} runs)",
              file=sys.stderr, flush=True)
    return rows


def _make(st, n, tau):
    """Storage names: fp64, fp32, fp16, bf16, and fp16sr / bf16sr for stochastic rounding."""
    return Lattice(n, n, n, tau=tau, storage=st[:4], stochastic=st.endswith("sr"), device="cuda:0")


def precision_study(n=512, steps=2000, every=100, storages=("fp64", "fp32", "fp16", "fp16sr", "bf16", "bf16sr")):
    wl = workloads.taylor_green(n, seed=1)
    lats = {}
    for st in storages:
        lat = _make(st, n, wl["tau"])
        lat.init(wl["rho"], wl["u"])
        lats[st] = lat
    del wl
    return lockstep(lats, steps, every, f"taylor_green_{n}")


def kolmogorov_study(n=384, steps=5000, every=500, storages=("fp64", "fp32", "fp16", "fp16sr")):
    wl = workloads.kolmogorov(n)
    lats = {}
    for st in storages:
        lat = _make(st, n, wl["tau"])
        lat.set_force("profile_y", wl["force_profile_y"])
        lat.init(wl["rho"], wl["u"])
        lats[st] = lat
    del wl
    return lockstep(lats, steps, every, f"kolmogorov_{n}")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["precision", "kolmogorov"])
    ap.add_argument("--n", type=int)
    ap.add_argument("--steps", type=int)
    ap.add_argument("--every", type=int)
    a = ap.parse_args(argv)
    kw = {k: v for k, v in (("n", a.n), ("steps", a.steps), ("every", a.every)) if v is not None}
    if a.study == "precision":
        precision_study(**kw)
    else:
        kolmogorov_study(**kw)


if __name__ == "__main__":
    main()
