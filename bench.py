"""Benchmark of the fused D3Q27 CM-LBM step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-fp16]

Headline workload: 3D Taylor-Green vortex, 256^3 periodic, FP32 populations,
u0 = 0.05, Re = 1600, zero force.  A step is one pass of the whole hot path
(one fused pull-stream + collide launch over every cell).  Prints one JSON line:
value = GLUPS (10^9 lattice-cell updates per second) of the timed K steps,
plus the HBM roofline of the step kernel, the FP16-storage variant at 512^3,
and the FP64 CPU oracle timed on the host cores on a bounded sample.
"""
import argparse
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
BYTES_PER_CELL = {"fp64": 432, "fp32": 216, "fp16": 108, "bf16": 108,  # 27 reads + 27 writes
                  "mom32": 72}  # moment representation: 9 FP32 numbers read + 9 written
# template arguments: storage, cells per lane, solid mask, force field, non-temporal stores, collision model,
# fused reductions
STEP_KERNEL = {"fp32": "k_step<1, 1, false, false, true, 0, false>", "fp16": "k_step<2, 2, false, false, true, 0, false>",
               "bf16": "k_step<3, 2, false, false, true, 0, false>", "fp64": "k_step<0, 1, false, false, true, 0, false>"}
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_step_tgv256_fp32_counters.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1905_10182_amd", "csrc", f) for f in ("cmlbm.hip", "d3q27.hpp")]


def source_digest():
    import hashlib
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if there is none or the kernel sources changed since it was taken."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    text = open(COUNTERS_FILE).read()
    m = re.search(r"source_digest:\s*([0-9a-f]+)", text)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != source_digest():
        return None
    return float(t.group(1))


def time_steps(lat, steps, warmup):
    import torch
    lat.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    lat.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3, wall


def run_gpu(n, storage, steps, warmup, stochastic=False):
    import workloads
    from paper_1905_10182_amd import Lattice

    wl = workloads.taylor_green(n, seed=1)
    lat = Lattice(n, n, n, tau=wl["tau"], storage=storage, stochastic=stochastic, device="cuda:0")
    lat.init(wl["rho"], wl["u"])
    del wl
    r0 = lat.reduce()
    secs, wall = time_steps(lat, steps, warmup)
    r1 = lat.reduce()
    ncell = n ** 3
    mass_drift = abs(r1[0, 0] / r0[0, 0] - 1)
    assert r1[0, 6] == 0, "non-finite state"
    lat.close()
    return dict(secs=secs, wall=wall, glups=ncell * steps / secs / 1e9, ms_per_step=secs / steps * 1e3,
                launch_s=secs / steps, bytes_per_launch=BYTES_PER_CELL[storage] * ncell, mass_drift=mass_drift,
                umax=float(r1[0, 5]))


# D2Q9 (App. B model): nine populations read + nine written, plus the force
# field (two components) read, per cell
BYTES_PER_CELL_2D = {"fp64": 144 + 16, "fp32": 72 + 8, "fp16": 36 + 8, "bf16": 36 + 8}
STEP_KERNEL_2D = {"fp64": "k2_step<0, 1, true>", "fp32": "k2_step<1, 2, true>", "fp16": "k2_step<2, 4, true>",
                  "bf16": "k2_step<3, 4, true>"}


def run_gpu_2d(n, storage, steps, warmup):
    """The four-rolls mill (App. B model, per-cell force field) on an n x n lattice."""
    import numpy as np
    import torch

    import workloads
    from paper_1905_10182_amd.cmlbm2d import Lattice2D

    wl = workloads.four_rolls_mill_2d(n, dtype=np.float32)
    lat = Lattice2D(n, n, tau=wl["tau"], storage=storage, device="cuda:0")
    lat.set_force("field", field=wl["force"])
    lat.init(np.ones(1, np.float32), wl["u_exact"], dtype=torch.float32)
    del wl
    secs, wall = time_steps(lat, steps, warmup)
    rho, u = lat.moments()
    finite = bool(torch.isfinite(u).all()) and bool(torch.isfinite(rho).all())
    assert finite, "non-finite state"
    mass_drift = abs(float(rho.sum()) / (n * n) - 1)
    del rho, u, lat
    torch.cuda.empty_cache()
    ncell = n * n
    return dict(secs=secs, wall=wall, glups=ncell * steps / secs / 1e9, ms_per_step=secs / steps * 1e3,
                launch_s=secs / steps, bytes_per_launch=BYTES_PER_CELL_2D[storage] * ncell, mass_drift=mass_drift)


# magnetic lattice (FP32): 21 populations read + 21 written, u (3 values) read
BYTES_PER_CELL_MHD = 21 * 4 * 2 + 12


def run_gpu_mhd(n, steps, warmup):
    """The magnetic lattice alone (FP32, n^3, periodic) stepped with a fixed
    velocity field: 21 populations read and written per cell plus u read."""
    import numpy as np
    import torch

    from paper_1905_10182_amd.mhd import MagneticLattice

    lat = MagneticLattice(n, n, n, 0.8, storage="fp32", device="cuda:0")
    c = torch.arange(n, device="cuda:0", dtype=torch.float32) * (2 * math.pi / n)
    z, y, x = torch.meshgrid(c, c, c, indexing="ij")
    b = torch.stack([torch.sin(y), torch.sin(z), torch.sin(x)]) * 0.01
    u = (torch.stack([torch.sin(z), torch.sin(x), torch.sin(y)]) * 0.02).contiguous()
    lat.init(b, u)
    del b, x, y, z
    for _ in range(warmup):
        lat.step(u)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        lat.step(u)
    e1.record(stream)
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / 1e3
    bf, _ = lat.fields()
    assert bool(torch.isfinite(bf).all()), "non-finite magnetic field"
    del lat, u, bf
    torch.cuda.empty_cache()
    ncell = n ** 3
    return dict(glups=ncell * steps / secs / 1e9, ms_per_step=secs / steps * 1e3,
                bytes_per_launch=BYTES_PER_CELL_MHD * ncell, launch_s=secs / steps)


def run_fused(n, calls):
    """cmlbm_step_reduce (a step whose kernel also forms the FP64 reductions of
    the state it reads) against cmlbm_reduce + cmlbm_step, wall clock per call
    (both wait for the stream), FP32 TGV n^3."""
    import torch
    import workloads
    from paper_1905_10182_amd import Lattice

    wl = workloads.taylor_green(n, seed=1)
    lat = Lattice(n, n, n, tau=wl["tau"], storage="fp32", fused_reduce=True, device="cuda:0")
    lat.init(wl["rho"], wl["u"])
    del wl
    lat.step(5)
    lat.step_reduce()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(calls):
        lat.step(1)
        torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / calls
    t0 = time.perf_counter()
    for _ in range(calls):
        r = lat.step_reduce()
    t_fused = (time.perf_counter() - t0) / calls
    t0 = time.perf_counter()
    for _ in range(calls):
        lat.reduce()
        lat.step(1)
        torch.cuda.synchronize()
    t_sep = (time.perf_counter() - t0) / calls
    lat.close()
    return {"workload": f"taylor_green_{n} fp32, one call per step, wall clock incl. the stream sync",
            "step_ms": round(t_step * 1e3, 4), "step_reduce_ms": round(t_fused * 1e3, 4),
            "reduce_then_step_ms": round(t_sep * 1e3, 4), "ke": float(r[0, 4])}


def copy_bandwidth():
    import torch
    n = 1 << 30  # 4 GiB of float32
    a = torch.empty(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 10
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3
    del a, b
    torch.cuda.empty_cache()
    return 2 * 4 * n * reps / s / 1e9


def kernel_copy_bandwidth():
    """Rate of the library's plain 16-byte non-temporal copy kernel on 4 GiB:
    the practical read + write ceiling of the device."""
    import torch
    from paper_1905_10182_amd.cmlbm import device_copy
    n = 1 << 30
    a = torch.empty(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    device_copy(b, a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 10
    for _ in range(reps):
        device_copy(b, a)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3
    del a, b
    torch.cuda.empty_cache()
    return 2 * 4 * n * reps / s / 1e9


def warm_start():
    """Steps to the 1e-8 residual for 64 held-out sphere channels (FP64
    solver) from rest and from the shipped U-Net's prediction."""
    from paper_1905_10182_amd import warmstart as ws

    net = ws.load_model()
    s = ws.evaluate(net, first_seed=1_000_000, nb=64, tol=1e-8, log=lambda m: print(f"[bench]   {m}", file=sys.stderr,
                                                                                    flush=True))
    r = s["results"]
    return {"workload": "64 channels 64x32x32, 1-4 spheres r 3-8, F_x ~ U[1e-6, 1e-5], tau 0.8, fp64, "
                        "seeds 1000000..1000063",
            "mean_steps_cold": r["cold"]["mean_steps"], "mean_steps_warm": r["warm"]["mean_steps"],
            "mean_steps_exact_moments": r["exact"]["mean_steps"],
            "speedup_steps": round(s["speedup_steps_warm"], 3), "speedup_wall": round(s["speedup_wall_warm"], 3),
            "speedup_steps_exact_moments": round(s["speedup_steps_exact"], 3),
            "prediction_rel_error_u": round(s["prediction_rel_error_u"], 5),
            "prediction_rel_error_rho": round(s["prediction_rel_error_rho"], 5),
            "warm_vs_cold_final_rel": s["warm_vs_cold_final_rel"], "inference_s": round(s["inference_seconds"], 4),
            "fallbacks": s["fallbacks"]}


def cpu_baseline():
    """The FP64 oracle (closed-form route, OpenMP) on a bounded sample of the
    same workload: Taylor-Green 128^3, 400 steps."""
    import oracle
    import workloads

    n, steps = 128, 400
    wl = workloads.taylor_green(n, seed=1)
    L = oracle.Lattice(n, n, n, tau=wl["tau"])
    L.init(wl["rho"], wl["u"])
    L.step(1)
    t0 = time.perf_counter()
    L.step(steps)
    s = time.perf_counter() - t0
    return {"value": n ** 3 * steps / s / 1e9, "unit": "GLUPS", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"taylor_green {n}^3 fp64, {steps} steps ({s:.1f} s)"}


def cpu_detail():
    """The oracle on the host cores in more detail (not part of the default run):
    closed-form route at 64^3 and 256^3 with one thread and with all threads,
    and the literal route (matrix algebra per cell) at 32^3."""
    import subprocess
    code = r"""
import json, os, sys, time
sys.path.insert(0, %r)
import oracle, workloads
def run(n, steps, variant):
    wl = workloads.taylor_green(n, seed=1)
    L = oracle.Lattice(n, n, n, tau=wl["tau"])
    L.init(wl["rho"], wl["u"])
    L.step(1, variant=variant)
    t0 = time.perf_counter()
    L.step(steps, variant=variant)
    s = time.perf_counter() - t0
    return {"n": n, "steps": steps, "route": variant, "threads": oracle.num_threads(), "mlups": round(n ** 3 * steps / s / 1e6, 3)}
for n, steps, v in ((64, 20, "closed"), (256, 3, "closed"), (32, 3, "literal")):
    print(json.dumps(run(n, steps, v)), flush=True)
""" % ROOT
    rows = []
    for threads in (1, os.cpu_count()):
        env = dict(os.environ, OMP_NUM_THREADS=str(threads))
        out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True)
        rows += [json.loads(l) for l in out.stdout.splitlines() if l.startswith("{")]
    model = ""
    try:
        model = next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"cpu_model": model, "cpu_count": os.cpu_count(), "runs": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp16", action="store_true", help="skip the FP16, BF16 and FP64 storage legs")
    ap.add_argument("--no-warmstart", action="store_true")
    ap.add_argument("--no-mom", action="store_true")
    ap.add_argument("--no-d2q9", action="store_true")
    ap.add_argument("--no-mhd", action="store_true")
    ap.add_argument("--cpu-detail", action="store_true", help="only time the oracle on the host in detail")
    ap.add_argument("--n", type=int, default=256)
    args = ap.parse_args()
    if args.cpu_detail:
        print(json.dumps(cpu_detail()), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the solver is single-GPU; "
              "a z-slab decomposition over several GPUs is not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "no GPU"
    print(f"[bench] TGV {args.n}^3 fp32: {args.warmup} warmup + {args.steps} timed steps", file=sys.stderr,
          flush=True)
    main_run = run_gpu(args.n, "fp32", args.steps, args.warmup)
    print(f"[bench] fp32 {main_run['glups']:.2f} GLUPS", file=sys.stderr, flush=True)
    extra = {}
    if not args.no_fp16:
        n16 = 512 if args.n == 256 else args.n
        print(f"[bench] TGV {n16}^3 fp16 storage", file=sys.stderr, flush=True)
        r16 = run_gpu(n16, "fp16", max(args.steps // 4, 10), max(args.warmup // 4, 5))
        extra["fp16_storage"] = {
            "workload": f"taylor_green_{n16} fp16-stored shifted populations, fp32 compute",
            "glups": round(r16["glups"], 3), "ms_per_step": round(r16["ms_per_step"], 4),
            "hbm_gbs": round(r16["bytes_per_launch"] / r16["launch_s"] / 1e9, 1),
            "hbm_frac": round(r16["bytes_per_launch"] / r16["launch_s"] / 1e9 / HBM_PEAK_GBS, 4),
            "speedup_vs_fp32_glups": round(r16["glups"] / main_run["glups"], 3)}
        print(f"[bench] fp16 {r16['glups']:.2f} GLUPS", file=sys.stderr, flush=True)
        r16s = run_gpu(n16, "fp16", max(args.steps // 4, 10), max(args.warmup // 4, 5), stochastic=True)
        extra["fp16_storage_stochastic_rounding"] = {
            "glups": round(r16s["glups"], 3), "ms_per_step": round(r16s["ms_per_step"], 4),
            "hbm_frac": round(r16s["bytes_per_launch"] / r16s["launch_s"] / 1e9 / HBM_PEAK_GBS, 4),
            "speedup_vs_fp32_glups": round(r16s["glups"] / main_run["glups"], 3)}
        print(f"[bench] fp16 stochastic rounding {r16s['glups']:.2f} GLUPS", file=sys.stderr, flush=True)
        print(f"[bench] TGV {n16}^3 bf16 storage", file=sys.stderr, flush=True)
        rb = run_gpu(n16, "bf16", max(args.steps // 4, 10), max(args.warmup // 4, 5))
        extra["bf16_storage"] = {
            "kernel": STEP_KERNEL["bf16"], "glups": round(rb["glups"], 3), "ms_per_step": round(rb["ms_per_step"], 4),
            "hbm_gbs": round(rb["bytes_per_launch"] / rb["launch_s"] / 1e9, 1),
            "hbm_frac": round(rb["bytes_per_launch"] / rb["launch_s"] / 1e9 / HBM_PEAK_GBS, 4),
            "speedup_vs_fp32_glups": round(rb["glups"] / main_run["glups"], 3)}
        print(f"[bench] bf16 {rb['glups']:.2f} GLUPS", file=sys.stderr, flush=True)
        print(f"[bench] TGV {args.n}^3 fp64 storage", file=sys.stderr, flush=True)
        r64 = run_gpu(args.n, "fp64", max(args.steps // 4, 10), max(args.warmup // 4, 5))
        extra["fp64_storage"] = {
            "workload": f"taylor_green_{args.n}, fp64 populations and arithmetic",
            "kernel": STEP_KERNEL["fp64"], "glups": round(r64["glups"], 3), "ms_per_step": round(r64["ms_per_step"], 4),
            "bytes_per_cell": BYTES_PER_CELL["fp64"],
            "hbm_gbs": round(r64["bytes_per_launch"] / r64["launch_s"] / 1e9, 1),
            "hbm_frac": round(r64["bytes_per_launch"] / r64["launch_s"] / 1e9 / HBM_PEAK_GBS, 4)}
        print(f"[bench] fp64 {r64['glups']:.2f} GLUPS", file=sys.stderr, flush=True)
    if not args.no_mom:
        for nm in sorted({args.n, 512 if args.n == 256 else args.n}):
            print(f"[bench] TGV {nm}^3 moment storage (FP32)", file=sys.stderr, flush=True)
            rm = run_gpu(nm, "mom32", args.steps if nm == args.n else max(args.steps // 4, 10),
                         args.warmup if nm == args.n else max(args.warmup // 4, 5))
            extra[f"moment_storage_{nm}"] = {
                "workload": f"taylor_green_{nm}, nine FP32 numbers per cell (rho - rho0, u, (1 - omega) k4..k8), "
                            "neighbour populations rebuilt in LDS",
                "glups": round(rm["glups"], 3), "ms_per_step": round(rm["ms_per_step"], 4),
                "bytes_per_cell": BYTES_PER_CELL["mom32"],
                "hbm_gbs": round(rm["bytes_per_launch"] / rm["launch_s"] / 1e9, 1),
                "speedup_vs_fp32_populations_256": round(rm["glups"] / main_run["glups"], 3),
                "mass_drift": rm["mass_drift"]}
            print(f"[bench] moment storage {nm}^3: {rm['glups']:.2f} GLUPS", file=sys.stderr, flush=True)
    if not args.no_d2q9:
        n2 = 8192
        res2 = {}
        for st in ("fp32", "fp16", "fp64"):
            print(f"[bench] D2Q9 four-rolls mill {n2}^2 {st}", file=sys.stderr, flush=True)
            r2 = run_gpu_2d(n2, st, max(args.steps // 2, 10), max(args.warmup // 2, 5))
            bw = r2["bytes_per_launch"] / r2["launch_s"] / 1e9
            res2[st] = {"glups": round(r2["glups"], 3), "ms_per_step": round(r2["ms_per_step"], 4),
                        "kernel": STEP_KERNEL_2D[st], "bytes_per_cell": BYTES_PER_CELL_2D[st],
                        "hbm_gbs": round(bw, 1), "hbm_frac": round(bw / HBM_PEAK_GBS, 4),
                        "mass_drift": r2["mass_drift"]}
            print(f"[bench] D2Q9 {st} {r2['glups']:.2f} GLUPS", file=sys.stderr, flush=True)
        extra["d2q9"] = {"workload": f"four_rolls_mill_2d_{n2} (App. B model, Re 100, u0 1e-3, per-cell force field)",
                         **res2}
    if not args.no_mhd:
        print("[bench] magnetic lattice 256^3 fp32", file=sys.stderr, flush=True)
        rmag = run_gpu_mhd(256, max(args.steps // 10, 10), 3)
        bw = rmag["bytes_per_launch"] / rmag["launch_s"] / 1e9
        extra["mhd_magnetic_lattice"] = {
            "workload": "D3Q7 vector populations (App. C), 256^3 periodic, fp32, fixed velocity field",
            "kernel": "k_mhd_step<float>", "glups": round(rmag["glups"], 3), "ms_per_step": round(rmag["ms_per_step"], 4),
            "bytes_per_cell": BYTES_PER_CELL_MHD, "hbm_gbs": round(bw, 1), "hbm_frac": round(bw / HBM_PEAK_GBS, 4)}
        print(f"[bench] magnetic lattice {rmag['glups']:.2f} GLUPS, {bw:.0f} GB/s", file=sys.stderr, flush=True)
    print(f"[bench] fused reductions, TGV {args.n}^3 fp32", file=sys.stderr, flush=True)
    extra["fused_reduce"] = run_fused(args.n, 20)
    extra["device_copy_gbs"] = round(copy_bandwidth(), 1)  # torch's copy
    extra["kernel_copy_gbs"] = round(kernel_copy_bandwidth(), 1)  # 16-byte non-temporal copy kernel
    if not args.no_warmstart:
        print("[bench] warm start: 64 sphere channels 64x32x32, cold vs U-Net init", file=sys.stderr, flush=True)
        extra["warm_start"] = warm_start()
    achieved = main_run["bytes_per_launch"] / main_run["launch_s"] / 1e9
    traffic = measured_traffic()
    cpu = None
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline()
    out = {
        "metric": "D3Q27 CM-LBM GLUPS & %HBM peak, FP32 vs FP16-store; warm-start speedup",
        "value": round(main_run["glups"], 4),
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_run["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"taylor_green_{args.n} periodic, fp32 populations, u0=0.05, Re=1600, "
                               f"zero force, seeded 1e-6 density noise", "cells": args.n ** 3,
                   "tau": round(3 * 0.05 * args.n / (2 * math.pi * 1600) + 0.5, 6)},
        "roofline": {"bound": "hbm", "kernel": STEP_KERNEL["fp32"], "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "bytes_per_cell": BYTES_PER_CELL["fp32"]},
        "cpu_baseline": cpu,
        "mass_drift": main_run["mass_drift"],
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
