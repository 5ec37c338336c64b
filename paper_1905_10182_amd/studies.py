"""Precision studies of the solver on one GPU.

    python -m paper_1905_10182_amd.studies precision [--n 512] [--steps 2000] [--every 100]
    python -m paper_1905_10182_amd.studies kolmogorov [--n 384] [--steps 5000] [--every 500]
    python -m paper_1905_10182_amd.studies four-rolls [--storage fp64] [--models m1,m4,m5] [--lattice d2q9]
    python -m paper_1905_10182_amd.studies stability [--n 128] [--steps 4000] [--every 200]
    python -m paper_1905_10182_amd.studies droplet [--n 200] [--steps 3000]
    python -m paper_1905_10182_amd.studies orszag-tang [--n 256] [--models m1,m5] [--current populations]
    python -m paper_1905_10182_amd.studies orszag-tang-3d [--n 64] [--models m1,m4,m5] [--re 100]
    python -m paper_1905_10182_amd.studies hartmann [--current populations|stencil]

``precision``: the 3D Taylor-Green vortex (u0 = 0.05, Re = 1600) advanced in
lockstep with FP64, FP32, FP16 and BF16 population storage (16-bit both with
round-to-nearest and with stochastic rounding), all resident on the GPU at
once.  At every checkpoint it reports the FP64-reduced kinetic energy of each
run and the relative L2 velocity error of each run against the FP64 and the
FP32 runs.

``kolmogorov``: Kolmogorov flow (F_x = F0 sin(2 pi 4 y / N), tau = 0.5005)
with FP64, FP32 and FP16 (both roundings) storage, same report.

``four-rolls``: convergence of the two-dimensional four-rolls mill (Re = 100,
one node in z, per-node force field) to its analytic steady state for
N = 8..256 at u0 = 1e-3 and 1e-2: relative L2 velocity error per grid and the
observed order between successive grids (the paper prints 1.998 for
u0 = 1e-3), for the method (m1) and optionally the comparison models m4
(second-order forcing) and m5 (second-order equilibrium and forcing).  Each
grid starts from the analytic field and runs for three relaxation times of
the box, 3 / (nu psi^2).  ``--lattice d2q9`` runs the same study on the
two-dimensional D2Q9 model of App. B (libcmlbm2d, the method only).

``stability``: the Taylor-Green vortex (u0 = 0.05) at Re = 1600, 10^4 and
10^5 with the method (m1) and the single-relaxation-time controls (bgk: the
classical BGK scheme with second-order equilibrium and Guo forcing; bgk6:
BGK with the complete equilibrium and forcing), FP32 storage: kinetic energy
at every checkpoint until the run ends or turns non-finite.

``droplet``: the static droplet of the pseudo-potential test (Shan-Chen force,
G = -6, 200^3, radius 40, tau = 2, tanh interface of width 8) with the
method (m1) and the comparison
models m4 and m5: mean kinetic energy over time, the force refreshed from the
density before every step (cmlbm_pseudopotential_force).

``orszag-tang``: the two-dimensional Orszag-Tang vortex of the MHD tests
(Sec. III): the D3Q27 fluid with one node in z coupled to the magnetic lattice
of App. C through the Lorentz force (libcmlbm_mhd), u = u0 (-sin y, sin x),
b = u0 (-sin y, sin 2x) on a 2 pi box, Ma = u0 / cs in {0.07, 0.14, 0.28},
Re = u0 (N / 2 pi) / nu = 1600, eta = nu, FP64.  Every 0.1 time units (in
units of (N / 2 pi) / u0 steps) it reports the kinetic energy relative to its
initial value and the peak current and vorticity in the same units.

``hartmann``: the Hartmann flow of the MHD tests (Sec. III) for Ha = 1, 3,
10, 20 and channel widths L = 8..128: error of the steady velocity against
the analytic profile and the observed order.

``orszag-tang-3d``: the three-dimensional Orszag-Tang vortex of Sec. III
(u0 = b0 = 0.0203, Re = 100 by default), peak current magnitude over time for
N = 32, 64, 128 (or the given N), stencil current.

All print one JSON object per checkpoint or grid.  Error norms are taken with torch
on device-resident moments (diagnostics only; the solver runs in libcmlbm).
"""
import argparse
import json
import sys
import time

import numpy as np

import workloads
from paper_1905_10182_amd.cmlbm import RED, Lattice
from paper_1905_10182_amd.cmlbm2d import Lattice2D


def _rel(a, b, torch):
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def lockstep(lattices, steps, every, label, out=sys.stdout, per_step_ke=False, ke_rows=None):
    """Advance the lattices together; every `every` steps print their velocity
    errors against the FP64 (and FP32) run and their FP64-reduced kinetic
    energy.  With per_step_ke (lattices created with fused reductions) the
    steps go through step_reduce and a row of every lattice's kinetic energy
    is printed for every step, at no extra pass over the populations (and
    appended to ke_rows if a list is given)."""
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
        if per_step_ke:
            for j in range(n):
                ke = {k: float(lattices[k].step_reduce(allow_unstable=True)[0][RED["ke"]]) for k in names}
                print(json.dumps({"study": label, "step": t + j, "ke": ke}), file=out, flush=True)
                if ke_rows is not None:
                    ke_rows.append({"step": t + j, **ke})
        else:
            for k in names:
                lattices[k].step(n)
        torch.cuda.synchronize()
        t += n
        print(f"[{label}] step {t} ({time.perf_counter() - t0:.2f} s for {n} steps x {len(names)} runs)",
              file=sys.stderr, flush=True)
    return rows


def _make(st, n, tau, fused=False):
    """Storage names: fp64, fp32, fp16, bf16, and fp16sr / bf16sr for stochastic rounding."""
    return Lattice(n, n, n, tau=tau, storage=st[:4], stochastic=st.endswith("sr"), fused_reduce=fused,
                   device="cuda:0")


def precision_study(n=512, steps=2000, every=100, storages=("fp64", "fp32", "fp16", "fp16sr", "bf16", "bf16sr"),
                    per_step_ke=False, re=1600.0):
    wl = workloads.taylor_green(n, re=re, seed=1)
    lats = {}
    for st in storages:
        lat = _make(st, n, wl["tau"], per_step_ke)
        lat.init(wl["rho"], wl["u"])
        lats[st] = lat
    del wl
    return lockstep(lats, steps, every, f"taylor_green_{n}", per_step_ke=per_step_ke)


def kolmogorov_study(n=384, steps=5000, every=500, storages=("fp64", "fp32", "fp16", "fp16sr"), per_step_ke=False):
    wl = workloads.kolmogorov(n)
    lats = {}
    for st in storages:
        lat = _make(st, n, wl["tau"], per_step_ke)
        lat.set_force("profile_y", wl["force_profile_y"])
        lat.init(wl["rho"], wl["u"])
        lats[st] = lat
    del wl
    return lockstep(lats, steps, every, f"kolmogorov_{n}", per_step_ke=per_step_ke)


def four_rolls_study(ns=(8, 16, 32, 64, 128, 256), u0s=(1e-3, 1e-2), relax=3.0, storage="fp64", models=("m1",),
                     out=sys.stdout):
    import math

    import numpy as np
    import torch

    rows = []
    for model, u0 in ((m, u) for m in models for u in u0s):
        prev = None
        for n in ns:
            wl = workloads.four_rolls_mill(n, u0=u0)
            lat = Lattice(n, n, 1, tau=wl["tau"], storage=storage, model=model, device="cuda:0")
            lat.set_force("field", field=wl["force"])
            lat.init(np.ones(wl["shape"]), wl["u_exact"])
            steps = int(relax * wl["t_relax"])
            t0 = time.perf_counter()
            lat.step(steps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            u = lat.moments()[1].double().cpu().numpy()
            ex = wl["u_exact"][:2]
            err = float(np.linalg.norm(u[:2] - ex) / np.linalg.norm(ex))
            row = {"study": "four_rolls_mill", "model": model, "storage": storage, "u0": u0, "n": n, "tau": wl["tau"],
                   "steps": steps, "error": err, "order": None if prev is None else math.log2(prev / err),
                   "seconds": round(dt, 2)}
            print(json.dumps(row), file=out, flush=True)
            rows.append(row)
            prev = err
            del lat
    return rows


def four_rolls_study_2d(ns=(8, 16, 32, 64, 128, 256), u0s=(1e-3, 1e-2), relax=3.0, storage="fp64",
                        out=sys.stdout):
    import math

    import torch

    rows = []
    for u0 in u0s:
        prev = None
        for n in ns:
            wl = workloads.four_rolls_mill_2d(n, u0=u0)
            lat = Lattice2D(n, n, tau=wl["tau"], storage=storage, device="cuda:0")
            lat.set_force("field", field=wl["force"])
            lat.init(np.ones(wl["shape"]), wl["u_exact"])
            steps = int(relax * wl["t_relax"])
            t0 = time.perf_counter()
            lat.step(steps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            u = lat.moments()[1].double().cpu().numpy()
            ex = wl["u_exact"]
            err = float(np.linalg.norm(u - ex) / np.linalg.norm(ex))
            row = {"study": "four_rolls_mill", "lattice": "d2q9", "model": "m1", "storage": storage, "u0": u0, "n": n,
                   "tau": wl["tau"], "steps": steps, "error": err,
                   "order": None if prev is None else math.log2(prev / err), "seconds": round(dt, 2)}
            print(json.dumps(row), file=out, flush=True)
            rows.append(row)
            prev = err
            del lat
    return rows


def orszag_tang_study(ns=(256,), mas=(0.07, 0.14, 0.28), models=("m1", "m5"), current="populations", re=1600.0,
                      tmax=2.0, every=0.1, storage="fp64", out=sys.stdout):
    import math

    import torch

    from paper_1905_10182_amd.mhd import CoupledMHD

    def ddx(f, axis):  # central difference on the periodic lattice
        return 0.5 * (torch.roll(f, -1, axis) - torch.roll(f, 1, axis))

    rows = []
    for n in ns:
        for ma in mas:
            u0 = ma / math.sqrt(3.0)
            nu = u0 * n / (2 * math.pi * re)
            tau, tau_m = 0.5 + 3 * nu, 0.5 + 4 * nu
            k = 2 * math.pi / n
            X, Y = np.meshgrid(np.arange(n), np.arange(n))
            u = np.zeros((3, 1, n, n))
            b = np.zeros((3, 1, n, n))
            u[0, 0], u[1, 0] = -u0 * np.sin(k * Y), u0 * np.sin(k * X)
            b[0, 0], b[1, 0] = -u0 * np.sin(k * Y), u0 * np.sin(2 * k * X)
            unit = n / (2 * math.pi * u0)  # steps per time unit
            for model in models:
                S = CoupledMHD(n, n, 1, tau, tau_m, storage=storage, model=model, current=current)
                S.init(np.ones((1, n, n)), u, b)
                ke0 = None
                t0 = time.perf_counter()
                for i in range(int(round(tmax / every)) + 1):
                    t = i * every
                    S.step(int(round(t * unit)) - S.time)
                    rho, uu, bb, jj = S.state()
                    ke = float((uu[:2] ** 2).sum())
                    ke0 = ke if ke0 is None else ke0
                    zeta = ddx(uu[1, 0], 1) - ddx(uu[0, 0], 0)
                    jst = ddx(bb[1, 0], 1) - ddx(bb[0, 0], 0)
                    finite = bool(torch.isfinite(uu).all())
                    row = {"study": "orszag_tang", "n": n, "ma": ma, "model": model, "current": current, "tau": tau,
                           "tau_m": tau_m, "t": round(t, 4), "step": S.time, "ke_rel": ke / ke0,
                           "jmax": float(jj[2].abs().max()) * unit, "jmax_stencil": float(jst.abs().max()) * unit,
                           "zeta_max": float(zeta.abs().max()) * unit, "finite": finite}
                    print(json.dumps(row), file=out, flush=True)
                    rows.append(row)
                    if not finite:
                        break
                print(f"[orszag-tang] N={n} Ma={ma} {model}: {S.time} steps in {time.perf_counter() - t0:.1f} s",
                      file=sys.stderr, flush=True)
                del S
    return rows


def orszag_tang_3d_study(ns=(32, 64, 128), re=100.0, models=("m1",), current="stencil", tmax=2.0, every=0.1,
                         storage="fp64", out=sys.stdout):
    """Three-dimensional Orszag-Tang vortex (Sec. III): u = u0 (-2 sin y,
    2 sin x, 0), b = 0.8 u0 (-2 sin 2y + sin z, 2 sin x + sin z, sin x + sin y)
    on a 2 pi box, u0 = 0.0203, Re = u0 (N / 2 pi) / nu, eta = nu; peak
    current magnitude and kinetic energy every `every` time units."""
    import math

    import torch

    from paper_1905_10182_amd.mhd import CoupledMHD

    def ddx(f, axis):
        return 0.5 * (torch.roll(f, -1, axis) - torch.roll(f, 1, axis))

    rows = []
    u0 = 0.0203
    for n in ns:
        nu = u0 * n / (2 * math.pi * re)
        tau, tau_m = 0.5 + 3 * nu, 0.5 + 4 * nu
        c = 2 * math.pi * np.arange(n) / n
        Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
        u = np.stack([-2 * u0 * np.sin(Y), 2 * u0 * np.sin(X), 0 * X])
        b = 0.8 * u0 * np.stack([-2 * np.sin(2 * Y) + np.sin(Z), 2 * np.sin(X) + np.sin(Z), np.sin(X) + np.sin(Y)])
        unit = n / (2 * math.pi * u0)
        for model in models:
            S = CoupledMHD(n, n, n, tau, tau_m, storage=storage, model=model, current=current)
            S.init(np.ones((1, n, n, n)), u[:, None], b[:, None])
            t_start = time.perf_counter()
            ke0 = None
            for i in range(int(round(tmax / every)) + 1):
                t = i * every
                S.step(int(round(t * unit)) - S.time)
                rho, uu, bb, jj = S.state()
                ke = float((uu ** 2).sum())
                ke0 = ke if ke0 is None else ke0
                # |curl b| by central differences (axes of bb: component, z, y, x)
                jx = ddx(bb[2], 1) - ddx(bb[1], 0)
                jy = ddx(bb[0], 0) - ddx(bb[2], 2)
                jz = ddx(bb[1], 2) - ddx(bb[0], 1)
                jmag = torch.sqrt(jx * jx + jy * jy + jz * jz)
                finite = bool(torch.isfinite(uu).all())
                row = {"study": "orszag_tang_3d", "n": n, "re": re, "model": model, "current": current, "tau": tau,
                       "t": round(t, 4), "step": S.time, "ke_rel": ke / ke0, "jmax": float(jmag.max()) * unit,
                       "finite": finite}
                print(json.dumps(row), file=out, flush=True)
                rows.append(row)
                if not finite:
                    break
            print(f"[orszag-tang-3d] N={n} Re={re} {model}: {S.time} steps in {time.perf_counter() - t_start:.1f} s",
                  file=sys.stderr, flush=True)
            del S
    return rows


def hartmann_study(Ls=(8, 16, 32, 64, 128), has=(1.0, 3.0, 10.0, 20.0), current="populations", nu=0.1, umax=1e-3,
                   storage="fp64", out=sys.stdout):
    """Hartmann flow (Sec. III): a channel of width L between halfway walls at
    which the field (0, B0, 0) is imposed, eta = nu, driven by a uniform force;
    relative L2 error of the steady velocity against
    u(s) = G a^2 / (nu Ha tanh Ha) [1 - cosh(Ha s / a) / cosh Ha] (a = L / 2,
    b_x = 0 at both walls), and the observed order between successive L."""
    import math

    from paper_1905_10182_amd.mhd import CoupledMHD

    rows = []
    for ha in has:
        prev = None
        for L in Ls:
            a = L / 2.0
            B0 = ha * nu / a
            G = umax * nu * ha * math.tanh(ha) / (a * a)
            b = np.zeros((3, 1, L, 1))
            b[1] = B0
            S = CoupledMHD(1, L, 1, 0.5 + 3 * nu, 0.5 + 4 * nu, storage=storage, current=current, wall=(0, 1, 0),
                           b_wall=(0.0, B0, 0.0), body_force=(G, 0.0, 0.0))
            S.init(np.ones((1, L, 1)), np.zeros((3, 1, L, 1)), b)
            # twelve e-foldings of the slowest mode: with eta = nu the Elsasser variables u +- b are
            # advected at +-B0 and diffuse with nu, rate nu (pi^2 + Ha^2) / (4 a^2)
            steps = int(48 * a * a / (nu * (math.pi ** 2 + ha * ha))) + 200
            t0 = time.perf_counter()
            S.step(steps)
            u = S.state()[1][0, 0, :, 0].double().cpu().numpy()
            s = np.arange(L) - (L - 1) / 2.0
            ua = G * a * a / (nu * ha * math.tanh(ha)) * (1 - np.cosh(ha * s / a) / math.cosh(ha))
            err = float(np.linalg.norm(u - ua) / np.linalg.norm(ua))
            row = {"study": "hartmann", "ha": ha, "L": L, "current": current, "steps": steps, "error": err,
                   "order": None if prev is None else math.log2(prev / err),
                   "seconds": round(time.perf_counter() - t0, 2)}
            print(json.dumps(row), file=out, flush=True)
            rows.append(row)
            prev = err
            del S
    return rows


def stability_study(n=128, res=(1600.0, 1e4, 1e5), models=("m1", "bgk", "bgk6"), steps=4000, every=200,
                    storage="fp32", out=sys.stdout):
    rows = []
    for re in res:
        wl = workloads.taylor_green(n, re=re, seed=1)
        for model in models:
            lat = Lattice(n, n, n, tau=wl["tau"], storage=storage, model=model, device="cuda:0")
            lat.init(wl["rho"], wl["u"])
            t, blew = 0, None
            while True:
                r = lat.reduce(allow_unstable=True)[0]
                row = {"study": "stability", "n": n, "re": re, "tau": wl["tau"], "model": model, "step": t,
                       "ke": float(r[RED["ke"]]), "umax": float(r[RED["umax"]]),
                       "nonfinite": int(r[RED["nonfinite"]])}
                print(json.dumps(row), file=out, flush=True)
                rows.append(row)
                if row["nonfinite"] > 0 or not row["umax"] < 1.0:
                    blew = t
                    break
                if t >= steps:
                    break
                lat.step(every)
                t += every
            print(f"[stability] n={n} Re={re:g} {model}: " + (f"blew up by step {blew}" if blew is not None
                  else f"stable for {steps} steps"), file=sys.stderr, flush=True)
            del lat
    return rows


def droplet_run(lat, wl, steps, out=sys.stdout, label="", every=lambda t: 10 if t < 500 else 50):
    """Advance a pseudo-potential lattice, refreshing the force field from the
    density before every step; report the mean kinetic energy at checkpoints.
    Returns (rows, step of blow-up or None)."""
    import torch

    dt = torch.float64 if lat.storage == 0 else torch.float32
    field = torch.zeros((3,) + lat.shape, dtype=dt, device=lat.device)
    lat.set_force("field", field=field)
    lat.init(wl["rho"], wl["u"])
    n = float(np.prod(lat.shape))
    rows, t, nxt = [], 0, 0
    rho = torch.empty(lat.shape, dtype=dt, device=lat.device)
    while True:
        lat.density(dtype=dt, out=rho)
        lat.pseudopotential_force(wl["g"], rho, out=field)
        if t == nxt:
            r = lat.reduce(allow_unstable=True)[0]
            row = {"study": "droplet", "label": label, "step": t, "ke_mean": float(r[RED["ke"]]) / n,
                   "umax": float(r[RED["umax"]]), "nonfinite": int(r[RED["nonfinite"]])}
            print(json.dumps(row), file=out, flush=True)
            rows.append(row)
            if row["nonfinite"] > 0 or not row["umax"] < 1.0:
                return rows, t
            nxt = t + every(t)
        if t >= steps:
            return rows, None
        lat.step(1)
        t += 1


def droplet_study(n=200, radius=40.0, models=("m1", "m4", "m5"), steps=3000, storage="fp64", out=sys.stdout):
    res = {}
    for model in models:
        wl = workloads.static_droplet(n, radius)
        lat = Lattice(n, n, n, tau=wl["tau"], storage=storage, model=model, device="cuda:0")
        rows, blew = droplet_run(lat, wl, steps, out=out, label=model)
        res[model] = (rows, blew)
        peak = max(r["ke_mean"] for r in rows if r["nonfinite"] == 0)
        print(f"[droplet] {model}: " + (f"non-finite by step {blew}" if blew is not None else f"stable to {steps}")
              + f", peak mean KE {peak:.3e}, final {rows[-1]['ke_mean']:.3e}", file=sys.stderr, flush=True)
        del lat
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["precision", "kolmogorov", "four-rolls", "stability", "droplet",
                                      "orszag-tang", "orszag-tang-3d", "hartmann"])
    ap.add_argument("--storage", default="fp64")
    ap.add_argument("--models", default="m1", help="comma-separated: m1 (the method), m4, m5, eq2")
    ap.add_argument("--lattice", default="d3q27", choices=["d3q27", "d2q9"])
    ap.add_argument("--current", default="populations", choices=["populations", "stencil"])
    ap.add_argument("--tmax", type=float, default=2.0)
    ap.add_argument("--re", type=float)
    ap.add_argument("--n", type=int)
    ap.add_argument("--steps", type=int)
    ap.add_argument("--every", type=int)
    ap.add_argument("--per-step-ke", action="store_true",
                    help="precision / kolmogorov: kinetic energy of every run at every step (fused reductions)")
    a = ap.parse_args(argv)
    kw = {k: v for k, v in (("n", a.n), ("steps", a.steps), ("every", a.every)) if v is not None}
    if a.study == "precision":
        precision_study(per_step_ke=a.per_step_ke, **kw)
    elif a.study == "kolmogorov":
        kolmogorov_study(per_step_ke=a.per_step_ke, **kw)
    elif a.study == "stability":
        stability_study(**kw)
    elif a.study == "orszag-tang":
        orszag_tang_study(ns=(a.n or 256,), models=tuple(a.models.split(",")), current=a.current, tmax=a.tmax)
    elif a.study == "hartmann":
        hartmann_study(current=a.current)
    elif a.study == "orszag-tang-3d":
        orszag_tang_3d_study(ns=(a.n,) if a.n else (32, 64, 128), re=a.re or 100.0,
                             models=tuple(a.models.split(",")), tmax=a.tmax)
    elif a.study == "droplet":
        droplet_study(storage=a.storage, **{k: v for k, v in kw.items() if k in ("n", "steps")})
    elif a.lattice == "d2q9":
        four_rolls_study_2d(storage=a.storage)
    else:
        four_rolls_study(storage=a.storage, models=tuple(a.models.split(",")))


if __name__ == "__main__":
    main()
