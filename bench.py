"""Benchmark of the fused D3Q27 CM-LBM step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--repeats R] [--legs LIST] [--error-steps E]
                    [--no-cpu] [--no-fp16] [--no-warmstart] [--no-mom] [--no-d2q9] [--no-mhd]
    python bench.py --cpu-detail

Headline workload: 3D Taylor-Green vortex, 256^3 periodic, FP32 populations,
u0 = 0.05, Re = 1600, zero force.  A step is one pass of the whole hot path
(one fused pull-stream + collide launch over every cell).  Every leg runs W
untimed warmup steps and then R timed windows of exactly K steps (HIP events
on the solver's stream, synchronised on both sides); its figure is the
median window.  Prints one JSON line: value = GLUPS (10^9 lattice-cell
updates per second) of the headline leg, the HBM roofline of its step
kernel, the FP64 CPU oracle timed on the host cores on a bounded sample,
and the other legs:
  - precision legs, Taylor-Green 512^3 (the same vortex, Re = 1600): FP64,
    FP32, FP16 and BF16 storage (16-bit with nearest and with stochastic
    rounding), each run first for E steps from the initial state with the
    fused reductions -- its kinetic energy at every step -- and compared
    after E steps with the FP64 run (relative L2 velocity error, eq. error
    of the paper) and with the FP32 run; then timed.  The 16-bit speed-ups
    are given against FP32 at the same size;
  - FP64 storage at 256^3, moment storage, the D2Q9 model, the magnetic
    lattice, the Shan-Chen droplet's coupled step, the fused reductions, copy
    kernels and the learned warm start.
"""
import argparse
import json
import math
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
BYTES_PER_CELL = {"fp64": 432, "fp32": 216, "fp16": 108, "bf16": 108,  # 27 reads + 27 writes
                  "mom32": 72}  # moment representation: 9 FP32 numbers read + 9 written
# template arguments: storage, cells per lane, solid mask, force field, non-temporal stores, collision model,
# fused reductions, stochastic rounding
STEP_KERNEL = {"fp32": "k_step<1, 1, false, false, true, 0, false, false>",
               "fp16": "k_step<2, 2, false, false, true, 0, false, false>",
               "fp16sr": "k_step<2, 2, false, false, true, 0, false, true>",
               "bf16": "k_step<3, 2, false, false, true, 0, false, false>",
               "bf16sr": "k_step<3, 2, false, false, true, 0, false, true>",
               "fp64": "k_step<0, 1, false, false, true, 0, false, false>"}
# committed rocprofv3 counter summary (FETCH_SIZE, WRITE_SIZE) of every step configuration
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_step_counters.md")
MOM_COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_step_mom_tgv_counters.md")
# non-packed FP32 VALU: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1905_10182_amd", "csrc", f) for f in ("cmlbm.hip", "d3q27.hpp")]
ALL_LEGS = ("fp32", "precision", "fp64", "mom", "d2q9", "mhd", "shanchen", "fused", "copy", "conv", "warmstart", "cpu")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


_RANGE = []


def mark(name):
    """Consecutive roctx ranges, one per leg (torch.cuda.nvtx is roctx on ROCm),
    so that a rocprofv3 --marker-trace of a bench run names each leg's kernels;
    None closes the last one."""
    import torch
    if _RANGE:
        torch.cuda.nvtx.range_pop()
        _RANGE.pop()
    if name:
        torch.cuda.nvtx.range_push(name)
        _RANGE.append(name)


def source_digest():
    import hashlib
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def counter_value(path, name, key):
    """A figure `name[key]` of a committed rocprofv3 counter summary, or None
    if there is none or the kernel sources changed since it was taken."""
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"source_digest:\s*([0-9a-f]+)", text)
    t = re.search(re.escape(name) + r"\[" + re.escape(key) + r"\]:\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != source_digest():
        return None
    return float(t.group(1))


def measured_traffic(key):
    """HBM bytes per launch of the step configuration `key`."""
    return counter_value(COUNTERS_FILE, "hbm_bytes_per_launch", key)


def alu_roofline(n, glups):
    """The moment kernel's VALU rate: its counted VALU lane-operations per
    cell (rocprofv3 SQ_INSTS_VALU x 64 / cells) times the measured cell rate,
    against the non-packed FP32 VALU peak; None without a current count."""
    v = counter_value(MOM_COUNTERS_FILE, "valu_lane_ops_per_cell", f"mom32_{n}")
    if v is None:
        return None
    a = v * glups * 1e9
    return {"bound": "alu", "kernel": "k_step_mom", "achieved": round(a / 1e12, 2), "peak": round(VALU_PEAK_LANE_OPS / 1e12, 2),
            "unit": "T lane-op/s", "frac": round(a / VALU_PEAK_LANE_OPS, 4), "valu_lane_ops_per_cell": v}


def time_steps(lat, steps, warmup, repeats):
    """warmup untimed steps, then `repeats` windows of exactly `steps` steps,
    each bracketed by a device synchronisation and timed with HIP events on the
    stream the solver launches on.  Returns the seconds of each window."""
    import torch
    lat.step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    out = []
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        lat.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1) / 1e3)
    return out


def rate(ncell, steps, windows, bytes_per_cell):
    """Figures of a timed leg from its windows (median window)."""
    secs = statistics.median(windows)
    launch = secs / steps
    gbs = bytes_per_cell * ncell / launch / 1e9
    return {"glups": round(ncell * steps / secs / 1e9, 4), "ms_per_step": round(launch * 1e3, 5),
            "window_ms_per_step": [round(w / steps * 1e3, 5) for w in windows],
            "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}


def run_gpu(n, storage, steps, warmup, repeats, stochastic=False, fields=None):
    """Time the step on the Taylor-Green vortex n^3 (FP32/FP64/16-bit/moment storage)."""
    import workloads
    from paper_1905_10182_amd import Lattice

    wl = fields or workloads.taylor_green(n, seed=1)
    lat = Lattice(n, n, n, tau=wl["tau"], storage=storage, stochastic=stochastic, device="cuda:0")
    lat.init(wl["rho"], wl["u"])
    del wl
    r0 = lat.reduce()
    windows = time_steps(lat, steps, warmup, repeats)
    r1 = lat.reduce()
    assert r1[0, 6] == 0, "non-finite state"
    lat.close()
    out = rate(n ** 3, steps, windows, BYTES_PER_CELL[storage])
    out["mass_drift"] = abs(r1[0, 0] / r0[0, 0] - 1)
    return out


def device_fields(n):
    """The Taylor-Green n^3 initial state uploaded once (FP64 on the device), reused by every leg."""
    import torch
    import workloads
    wl = workloads.taylor_green(n, seed=1)
    return {"tau": wl["tau"], "rho": torch.as_tensor(wl["rho"], device="cuda:0"),
            "u": torch.as_tensor(wl["u"], device="cuda:0")}


def precision_legs(n, names, steps, warmup, repeats, error_steps, fields):
    """Each configuration from the same initial state: error_steps steps through
    cmlbm_step_reduce (kinetic energy of every step), velocity after them
    compared with the FP64 and FP32 runs, then the timed windows."""
    import torch
    from paper_1905_10182_amd import Lattice

    ref = {}
    ke_ref = {}
    out = {}
    for name in names:
        st, sr = name[:4], name.endswith("sr")
        log(f"TGV {n}^3 {name}: {error_steps} steps with per-step kinetic energy")
        lat = Lattice(n, n, n, tau=fields["tau"], storage=st, stochastic=sr, fused_reduce=True, device="cuda:0")
        lat.init(fields["rho"], fields["u"])
        t0 = time.perf_counter()
        ke = [float(lat.step_reduce(allow_unstable=True)[0, 4]) for _ in range(error_steps)]
        t_err = time.perf_counter() - t0
        u = lat.moments(dtype=torch.float64)[1]
        finite = bool(torch.isfinite(u).all())
        row = {"kernel": STEP_KERNEL[name], "rounding": "stochastic" if sr else ("nearest" if st in ("fp16", "bf16")
                                                                                  else None)}
        err = {"steps": error_steps, "finite": finite}
        for rk in ("fp64", "fp32"):
            if rk in ref and rk != name:
                err[f"rel_l2_u_vs_{rk}"] = float(torch.linalg.vector_norm(u - ref[rk]) /
                                                 torch.linalg.vector_norm(ref[rk]))
                err[f"max_rel_ke_dev_vs_{rk}"] = max(abs(a / b - 1) for a, b in zip(ke, ke_ref[rk]))
        err["ke_final"] = ke[-1]
        row["error"] = err
        if name in ("fp64", "fp32"):
            ref[name] = u
            ke_ref[name] = ke
        else:
            del u
        log(f"  {name}: {err} ({t_err:.1f} s)")
        if name != "fp64":  # FP64 storage is timed at the headline size
            windows = time_steps(lat, steps, warmup, repeats)
            row.update(rate(n ** 3, steps, windows, BYTES_PER_CELL[st]))
            row["traffic"] = measured_traffic(name)
            log(f"  {name}: {row['glups']:.2f} GLUPS, {row['hbm_gbs']:.0f} GB/s")
        lat.close()
        torch.cuda.empty_cache()
        out[name] = row
    del ref
    torch.cuda.empty_cache()
    return out


# D2Q9 (App. B model): nine populations read + nine written, plus the force
# field (two components) read, per cell
BYTES_PER_CELL_2D = {"fp64": 144 + 16, "fp32": 72 + 8, "fp16": 36 + 8, "bf16": 36 + 8}
STEP_KERNEL_2D = {"fp64": "k2_step<0, 1, true>", "fp32": "k2_step<1, 2, true>", "fp16": "k2_step<2, 4, true>",
                  "bf16": "k2_step<3, 4, true>"}


def run_gpu_2d(n, storage, steps, warmup, repeats):
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
    windows = time_steps(lat, steps, warmup, repeats)
    rho, u = lat.moments()
    finite = bool(torch.isfinite(u).all()) and bool(torch.isfinite(rho).all())
    assert finite, "non-finite state"
    mass_drift = abs(float(rho.sum()) / (n * n) - 1)
    del rho, u, lat
    torch.cuda.empty_cache()
    out = rate(n * n, steps, windows, BYTES_PER_CELL_2D[storage])
    out.update(kernel=STEP_KERNEL_2D[storage], bytes_per_cell=BYTES_PER_CELL_2D[storage], mass_drift=mass_drift)
    return out


# magnetic lattice (FP32): 21 populations read + 21 written, u (3 values) read
BYTES_PER_CELL_MHD = 21 * 4 * 2 + 12


def run_shan_chen(n, radius, steps, warmup, repeats):
    """The static droplet's coupled step at n^3 in FP32 (G = -6, tau 2):
    the density from the moment export, the Shan-Chen force from it
    (k_pseudopotential), then the fused step with that force field; and the
    force kernel alone, whose algorithmic traffic is the density read once and
    the three force components written, 16 B per cell; and the density export
    alone (k_gather with no velocity: 27 FP32 populations read, the density
    written, 112 B per cell)."""
    import torch

    import workloads
    from paper_1905_10182_amd import Lattice
    from paper_1905_10182_amd.cmlbm import RED

    wl = workloads.static_droplet(n, radius)
    lat = Lattice(n, n, n, tau=wl["tau"], storage="fp32", device="cuda:0")
    field = torch.zeros((3,) + lat.shape, dtype=torch.float32, device="cuda:0")
    lat.set_force("field", field=field)
    lat.init(wl["rho"], wl["u"])
    g = wl["g"]
    del wl

    rho = torch.empty(lat.shape, dtype=torch.float32, device="cuda:0")

    def coupled():
        lat.density(dtype=torch.float32, out=rho)
        lat.pseudopotential_force(g, rho, out=field)
        lat.step(1)

    def timed(fn, count):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        ws = []
        for _ in range(repeats):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(count):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ws.append(e0.elapsed_time(e1) / 1e3 / count)
        return statistics.median(ws)

    t_step = timed(coupled, steps)
    lat.density(dtype=torch.float32, out=rho)
    t_force = timed(lambda: lat.pseudopotential_force(g, rho, out=field), 20)
    t_dens = timed(lambda: lat.density(dtype=torch.float32, out=rho), 20)
    red = lat.reduce(allow_unstable=True)
    cells = n ** 3
    gbs = 16.0 * cells / t_force / 1e9
    dgbs = 112.0 * cells / t_dens / 1e9
    out = {"workload": f"static_droplet_{n} (radius {radius:g}, G = -6, tau 2), fp32; per coupled step: density "
                       "export, pseudo-potential force, fused step", "steps_run": warmup + repeats * steps,
           "finite": bool(red[0, RED["nonfinite"]] == 0), "ms_per_coupled_step": round(t_step * 1e3, 4),
           "glups_coupled": round(cells / t_step / 1e9, 3), "force_kernel": "k_pseudopotential<float>",
           "force_us": round(t_force * 1e6, 1), "force_bytes_per_cell": 16, "force_hbm_gbs": round(gbs, 1),
           "force_hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "density_kernel": "k_gather<1, false>",
           "density_us": round(t_dens * 1e6, 1), "density_bytes_per_cell": 112,
           "density_hbm_gbs": round(dgbs, 1), "density_hbm_frac": round(dgbs / HBM_PEAK_GBS, 4)}
    del lat, field, rho
    torch.cuda.empty_cache()
    return out


def run_gpu_mhd(n, steps, warmup, repeats):
    """The magnetic lattice alone (FP32, n^3, periodic) stepped with a fixed
    velocity field: 21 populations read and written per cell plus u read."""
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
    windows = []
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            lat.step(u)
        e1.record(stream)
        torch.cuda.synchronize()
        windows.append(e0.elapsed_time(e1) / 1e3)
    bf, _ = lat.fields()
    assert bool(torch.isfinite(bf).all()), "non-finite magnetic field"
    del lat, u, bf
    torch.cuda.empty_cache()
    out = rate(n ** 3, steps, windows, BYTES_PER_CELL_MHD)
    out.update(kernel="k_mhd_step<float>", bytes_per_cell=BYTES_PER_CELL_MHD)
    return out


def run_fused(n, calls, fields):
    """cmlbm_step_reduce (a step whose kernel also forms the FP64 reductions of
    the state it reads) against cmlbm_reduce + cmlbm_step, wall clock per call
    (both wait for the stream), FP32 TGV n^3."""
    import torch
    from paper_1905_10182_amd import Lattice

    lat = Lattice(n, n, n, tau=fields["tau"], storage="fp32", fused_reduce=True, device="cuda:0")
    lat.init(fields["rho"], fields["u"])
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


BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 MFMA


def run_conv(steps, warmup, repeats):
    """The learned part's kernels: Adam training steps of the warm-start U-Net
    (batch 16 x 32 x 32 x 64 voxels, forward + masked MSE + backward + Adam, all
    in libcmnn) on synthetic inputs and targets, and the three convolution
    kernels alone on one layer of each resolution level, against the dense
    BF16 MFMA peak."""
    import numpy as np
    import torch
    from paper_1905_10182_amd import cmnn
    from paper_1905_10182_amd import warmstart as ws
    from paper_1905_10182_amd.unet import UNet3D

    g = np.random.Generator(np.random.PCG64(2024))
    nb, batch = 32, 16
    shape = (nb, ws.NZ, ws.NY, ws.NX)
    data = {"x": g.uniform(0, 1, (nb, 2) + shape[1:]).astype(np.float32),
            "y": g.normal(0, 0.1, (nb, ws.NOUT) + shape[1:]).astype(np.float32),
            "w": (g.uniform(0, 1, shape) > 0.1).astype(np.float32)}
    net = UNet3D((ws.NZ, ws.NY, ws.NX), out_ch=ws.NOUT, seed=0)
    tr = ws.Trainer(net, data, batch=batch)
    for _ in range(warmup):
        tr.step(1e-4)
    torch.cuda.synchronize()
    windows = []
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            tr.step(1e-4)
        e1.record()
        torch.cuda.synchronize()
        windows.append(e0.elapsed_time(e1) / 1e3)
    secs = statistics.median(windows) / steps
    flops = 3 * net.flops_per_sample() * batch
    out = {"workload": f"U-Net training step, batch {batch} x 32 x 32 x 64, {net.nparams_real} parameters, "
                       "synthetic inputs", "ms_per_step": round(secs * 1e3, 4),
           "conv_tflops": round(flops / secs / 1e12, 1), "layers": {}}
    del tr, net, data
    torch.cuda.empty_cache()
    dev = "cuda:0"
    for name, dims, cin, cout in (("level0_32x32", (batch, 32, 32, 64), 32, 32),
                                  ("level1_64x64", (batch, 16, 16, 32), 64, 64),
                                  ("level2_64x96", (batch, 8, 8, 16), 64, 96)):
        geo = cmnn.geom(*dims, periodic=(1, 0, 1))
        x = torch.randn(dims + (cin,), device=dev).to(torch.bfloat16)
        dy = torch.randn(dims + (cout,), device=dev).to(torch.bfloat16)
        wf = (0.05 * torch.randn((27, cout, cin), device=dev)).to(torch.bfloat16)
        wt = wf.transpose(1, 2).contiguous()
        y = torch.empty(dims + (cout,), dtype=torch.bfloat16, device=dev)
        dx = torch.empty(dims + (cin,), dtype=torch.bfloat16, device=dev)
        dw = torch.empty((27, cout, cin), dtype=torch.float32, device=dev)
        wsp = torch.empty(cmnn.conv_bwd_weight_workspace(geo, cin, cout) // 4, dtype=torch.float32, device=dev)
        ops = {"fwd": lambda: cmnn.conv_fwd(geo, x, cin, wf, None, cout, cmnn.ACT_NONE, y),
               "bwd_data": lambda: cmnn.conv_bwd_data(geo, dy, cout, wt, cin, dx),
               "bwd_weight": lambda: cmnn.conv_bwd_weight(geo, x, cin, dy, cout, dw, None, wsp)}
        fl = 2.0 * 27 * cin * cout * int(np.prod(dims))
        row = {"dims": list(dims), "cin": cin, "cout": cout, "gflop": round(fl / 1e9, 2)}
        for op, fn in ops.items():
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(repeats):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(20):
                    fn()
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1) / 1e3 / 20)
            t = statistics.median(ts)
            row[op] = {"us": round(t * 1e6, 1), "tflops": round(fl / t / 1e12, 1),
                       "frac_bf16_peak": round(fl / t / 1e12 / BF16_PEAK_TFLOPS, 4)}
        out["layers"][name] = row
        del x, dy, wf, wt, y, dx, dw, wsp
        torch.cuda.empty_cache()
    return out


def pattern_copy_rate(n=256, repeats=5, launches=20):
    """The FP32 step's memory traffic without its arithmetic on the headline
    lattice's layout (n^2 lattice rows, each a block of 27 population rows of
    n cells): median of `repeats` windows of `launches` row-block copies."""
    import torch
    from paper_1905_10182_amd import cmlbm
    assert (4 * n) % 256 == 0  # rows are whole 256-byte lines, so a population row is n values
    cells = n ** 3
    a = torch.zeros(27 * cells, dtype=torch.float32, device="cuda:0")
    b = torch.zeros_like(a)
    for _ in range(3):
        cmlbm.row_block_copy(b, a, n * n, n)
    torch.cuda.synchronize()
    ts = []
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(launches):
            cmlbm.row_block_copy(b, a, n * n, n)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) / launches)
    ms = statistics.median(ts)
    del a, b
    torch.cuda.empty_cache()
    return {"workload": f"{n}^3 FP32 cells, 27 population rows per lattice row in, 27 out, one cell per lane, "
                        "no arithmetic",
            "ms_per_launch": round(ms, 5), "gbs": round(2 * 27 * 4 * cells / (ms * 1e-3) / 1e9, 1)}


def copy_bandwidth(fn):
    """Read + write rate of fn(dst, src) on 4 GiB, median of 10 calls."""
    import torch
    n = 1 << 30
    a = torch.empty(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    fn(b, a)
    torch.cuda.synchronize()
    ts = []
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn(b, a)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    del a, b
    torch.cuda.empty_cache()
    return 2 * 4 * n / statistics.median(ts) / 1e9


def warm_start():
    """Steps to the 1e-8 residual for 64 held-out sphere channels (FP64
    solver) from rest and from the shipped U-Net's prediction."""
    from paper_1905_10182_amd import warmstart as ws

    net = ws.load_model()
    s = ws.evaluate(net, first_seed=1_000_000, nb=64, tol=1e-8, log=lambda m: log(f"  {m}"))
    r = s["results"]
    rnd = lambda v, k=3: None if v is None else round(v, k)  # noqa: E731
    return {"workload": "64 channels 64x32x32, 1-4 spheres r 3-8, F_x ~ U[1e-6, 1e-5], tau 0.8, fp64, "
                        "seeds 1000000..1000063",
            "mean_steps_cold": r["cold"]["mean_steps"], "mean_steps_warm": r["warm"]["mean_steps"],
            "mean_steps_exact_moments": r["exact"]["mean_steps"],
            "all_converged": all(v["all_converged"] for v in r.values()),
            "speedup_steps": rnd(s["speedup_steps_warm"]), "speedup_wall": rnd(s["speedup_wall_warm"]),
            "speedup_steps_exact_moments": rnd(s["speedup_steps_exact"]),
            "prediction_rel_error_u": round(s["prediction_rel_error_u"], 5),
            "prediction_rel_error_rho": round(s["prediction_rel_error_rho"], 5),
            "warm_vs_cold_final_rel": s["warm_vs_cold_final_rel"], "inference_s": round(s["inference_seconds"], 4),
            "fallbacks": s["fallbacks"], "fallback_reasons": s["fallback_reasons"]}


_ORACLE_RUN = r"""
import json, sys, time
sys.path.insert(0, %r)
import oracle, workloads
n, steps, variant = %d, %d, %r
wl = workloads.taylor_green(n, seed=1)
L = oracle.Lattice(n, n, n, tau=wl["tau"])
L.init(wl["rho"], wl["u"])
del wl
L.step(1, variant=variant)
t0 = time.perf_counter()
L.step(steps, variant=variant)
s = time.perf_counter() - t0
print(json.dumps({"n": n, "steps": steps, "route": variant, "threads": oracle.num_threads(), "seconds": s,
                  "glups": n ** 3 * steps / s / 1e9}), flush=True)
"""


def oracle_rate(n, steps, threads=None, variant="closed"):
    """The FP64 oracle (closed-form route, OpenMP) timed in a child process
    (its thread count is fixed when the OpenMP runtime starts)."""
    import subprocess
    env = dict(os.environ)
    if threads:
        env["OMP_NUM_THREADS"] = str(threads)
    res = subprocess.run([sys.executable, "-c", _ORACLE_RUN % (ROOT, n, steps, variant)], env=env,
                         capture_output=True, text=True, check=True)
    return json.loads([l for l in res.stdout.splitlines() if l.startswith("{")][-1])


def cpu_baseline():
    """The FP64 oracle on the headline workload itself (Taylor-Green 256^3): a
    bounded sample of 8 steps on all host threads and 1 step on one thread."""
    allc = oracle_rate(256, 8)
    one = oracle_rate(256, 1, threads=1)
    return {"value": round(allc["glups"], 5), "unit": "GLUPS", "cores": allc["threads"], "kind": "oracle",
            "sample": f"taylor_green 256^3 fp64 closed-form route: {allc['steps']} steps on {allc['threads']} "
                      f"threads ({allc['seconds']:.1f} s); 1 step on 1 thread ({one['seconds']:.1f} s)",
            "one_thread_glups": round(one["glups"], 5)}


def cpu_detail():
    """The oracle on the host cores in more detail (not part of the default run):
    closed-form route at 64^3 and 256^3 with one thread and with all threads,
    and the literal route (matrix algebra per cell) at 32^3."""
    rows = []
    for threads in (1, os.cpu_count()):
        for n, steps, v in ((64, 20, "closed"), (256, 3, "closed"), (32, 3, "literal")):
            r = oracle_rate(n, steps, threads, v)
            r["mlups"] = round(r.pop("glups") * 1e3, 3)
            rows.append(r)
    model = ""
    try:
        model = next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"cpu_model": model, "cpu_count": os.cpu_count(), "runs": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--repeats", type=int, default=3)
    ap.add_argument("--legs", default=",".join(ALL_LEGS), help=f"comma-separated subset of {','.join(ALL_LEGS)}")
    ap.add_argument("--precision", default="fp64,fp32,fp16,fp16sr,bf16,bf16sr",
                    help="configurations of the precision legs")
    ap.add_argument("--error-steps", type=int, default=2000)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--n16", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp16", action="store_true", help="skip the precision legs and the FP64 storage leg")
    ap.add_argument("--no-warmstart", action="store_true")
    ap.add_argument("--no-mom", action="store_true")
    ap.add_argument("--no-d2q9", action="store_true")
    ap.add_argument("--no-mhd", action="store_true")
    ap.add_argument("--cpu-detail", action="store_true", help="only time the oracle on the host in detail")
    args = ap.parse_args()
    if args.cpu_detail:
        print(json.dumps(cpu_detail()), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the solver is single-GPU; "
              "a z-slab decomposition over several GPUs is not built.", file=sys.stderr)
        sys.exit(2)
    legs = set(args.legs.split(","))
    for flag, leg in (("no_cpu", "cpu"), ("no_warmstart", "warmstart"), ("no_mom", "mom"), ("no_d2q9", "d2q9"),
                      ("no_mhd", "mhd")):
        if getattr(args, flag):
            legs.discard(leg)
    if args.no_fp16:
        legs -= {"precision", "fp64"}
    K, W, R = args.steps, args.warmup, args.repeats

    import torch
    assert torch.cuda.is_available(), "no GPU"
    n = args.n
    fields = device_fields(n)
    main_run = None
    extra = {}
    if "fp32" in legs:
        mark("fp32")
        log(f"TGV {n}^3 fp32: {W} warmup + {R} x {K} timed steps")
        main_run = run_gpu(n, "fp32", K, W, R, fields=fields)
        log(f"fp32 {main_run['glups']:.2f} GLUPS ({main_run['window_ms_per_step']} ms per step)")
    if "fp64" in legs:
        mark("fp64")
        log(f"TGV {n}^3 fp64 storage")
        r64 = run_gpu(n, "fp64", K, W, R, fields=fields)
        extra["fp64_storage"] = {"workload": f"taylor_green_{n}, fp64 populations and arithmetic",
                                 "kernel": STEP_KERNEL["fp64"], "bytes_per_cell": BYTES_PER_CELL["fp64"],
                                 "traffic": measured_traffic("fp64"), **r64}
        log(f"fp64 {r64['glups']:.2f} GLUPS")
    if "fused" in legs:
        mark("fused")
        log(f"fused reductions, TGV {n}^3 fp32")
        extra["fused_reduce"] = run_fused(n, 20, fields)
    if "mom" in legs:
        mark("mom")
        log(f"TGV {n}^3 moment storage (FP32)")
        rm = run_gpu(n, "mom32", K, W, R, fields=fields)
        extra[f"moment_storage_{n}"] = {
            "workload": f"taylor_green_{n}, nine FP32 numbers per cell (rho - rho0, u, (1 - omega) k4..k8), "
                        "neighbour populations rebuilt in LDS", "bytes_per_cell": BYTES_PER_CELL["mom32"], **rm,
            "roofline": alu_roofline(n, rm["glups"])}
        log(f"moment storage {n}^3: {rm['glups']:.2f} GLUPS")
    del fields
    torch.cuda.empty_cache()
    n16 = args.n16
    if "precision" in legs or ("mom" in legs and n16 != n):
        f16 = device_fields(n16)
        if "precision" in legs:
            mark("precision")
            names = [s for s in args.precision.split(",") if s]
            prec = precision_legs(n16, names, K, W, R, args.error_steps, f16)
            ref32 = prec.get("fp32", {}).get("glups")
            for name, row in prec.items():
                if ref32 and name != "fp32" and "glups" in row:
                    row["speedup_vs_fp32_same_size"] = round(row["glups"] / ref32, 3)
                if main_run and "glups" in row:
                    row[f"speedup_vs_fp32_{n}"] = round(row["glups"] / main_run["glups"], 3)
            extra["precision"] = {
                "workload": f"taylor_green_{n16} periodic, u0=0.05, Re=1600, seeded 1e-6 density noise; every "
                            f"configuration from the same initial state; errors after {args.error_steps} steps",
                **prec}
            target = prec.get("fp16sr")
            if target and "speedup_vs_fp32_same_size" in target:
                e = target["error"].get("rel_l2_u_vs_fp64")
                extra["fp16_target"] = {
                    "configuration": "fp16 storage, stochastic rounding",
                    "speedup_vs_fp32_same_size": target["speedup_vs_fp32_same_size"],
                    "rel_l2_u_vs_fp64": e, "steps": args.error_steps,
                    "meets_1.7x_at_1e-3": bool(target["speedup_vs_fp32_same_size"] >= 1.7 and e is not None
                                               and e <= 1e-3)}
        if "mom" in legs and n16 != n:
            mark(f"mom_{n16}")
            log(f"TGV {n16}^3 moment storage (FP32)")
            rm = run_gpu(n16, "mom32", K, W, R, fields=f16)
            extra[f"moment_storage_{n16}"] = {"bytes_per_cell": BYTES_PER_CELL["mom32"], **rm,
                                              "roofline": alu_roofline(n16, rm["glups"])}
            log(f"moment storage {n16}^3: {rm['glups']:.2f} GLUPS")
        del f16
        torch.cuda.empty_cache()
    if "d2q9" in legs:
        mark("d2q9")
        n2 = 8192
        res2 = {}
        for st in ("fp32", "fp16", "fp64"):
            log(f"D2Q9 four-rolls mill {n2}^2 {st}")
            res2[st] = run_gpu_2d(n2, st, K, W, R)
            log(f"D2Q9 {st} {res2[st]['glups']:.2f} GLUPS")
        extra["d2q9"] = {"workload": f"four_rolls_mill_2d_{n2} (App. B model, Re 100, u0 1e-3, per-cell force field)",
                         **res2}
    if "mhd" in legs:
        mark("mhd")
        log("magnetic lattice 256^3 fp32")
        rmag = run_gpu_mhd(256, K, W, R)
        extra["mhd_magnetic_lattice"] = {
            "workload": "D3Q7 vector populations (App. C), 256^3 periodic, fp32, fixed velocity field", **rmag}
        log(f"magnetic lattice {rmag['glups']:.2f} GLUPS")
    if "shanchen" in legs:
        mark("shanchen")
        log("Shan-Chen droplet 200^3 fp32, coupled step")
        extra["shan_chen"] = run_shan_chen(200, 40.0, max(K // 4, 10), max(W // 4, 2), R)
        log(f"Shan-Chen coupled step {extra['shan_chen']['ms_per_coupled_step']} ms, force kernel "
            f"{extra['shan_chen']['force_hbm_gbs']} GB/s")
    if "copy" in legs:
        mark("copy")
        from paper_1905_10182_amd.cmlbm import device_copy
        extra["device_copy_gbs"] = round(copy_bandwidth(lambda b, a: b.copy_(a)), 1)  # torch's copy
        extra["kernel_copy_gbs"] = round(copy_bandwidth(device_copy), 1)  # 16-byte non-temporal copy kernel
        extra["pattern_copy"] = pattern_copy_rate()  # the FP32 step's access pattern without arithmetic
    if "conv" in legs:
        mark("conv")
        log("U-Net training steps and convolution kernels (libcmnn)")
        extra["conv"] = run_conv(max(K // 10, 5), max(W // 10, 2), R)
        log(f"U-Net training step {extra['conv']['ms_per_step']} ms, {extra['conv']['conv_tflops']} TFLOP/s")
    if "warmstart" in legs:
        mark("warmstart")
        log("warm start: 64 sphere channels 64x32x32, cold vs U-Net init")
        extra["warm_start"] = warm_start()
    mark(None)
    cpu = None
    if "cpu" in legs:
        log("cpu baseline (oracle, taylor_green 256^3)")
        cpu = cpu_baseline()
    out = {
        "metric": "D3Q27 CM-LBM GLUPS & %HBM peak, FP32 vs FP16-store; warm-start speedup",
        "value": main_run["glups"] if main_run else None,
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "repeats": R,
        "ms_per_step": main_run["ms_per_step"] if main_run else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"taylor_green_{n} periodic, fp32 populations, u0=0.05, Re=1600, "
                               f"zero force, seeded 1e-6 density noise", "cells": n ** 3,
                   "tau": round(3 * 0.05 * n / (2 * math.pi * 1600) + 0.5, 6)},
        "roofline": None if main_run is None else {
            "bound": "hbm", "kernel": STEP_KERNEL["fp32"], "achieved": main_run["hbm_gbs"], "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": main_run["hbm_frac"], "traffic": measured_traffic("fp32"),
            "bytes_per_cell": BYTES_PER_CELL["fp32"], "window_ms_per_step": main_run["window_ms_per_step"],
            "source_digest": source_digest(),
            # the same row-block access pattern with no arithmetic, timed in this run (copy leg)
            "pattern_copy_gbs": extra["pattern_copy"]["gbs"] if "pattern_copy" in extra else None},
        "cpu_baseline": cpu,
        "mass_drift": main_run["mass_drift"] if main_run else None,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
