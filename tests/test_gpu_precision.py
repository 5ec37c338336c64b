"""Precision of 16-bit population storage over many steps, through the
lockstep driver of the precision study (studies.lockstep): the Taylor-Green
vortex 64^3 (u0 = 0.05, Re = 200: the same tau = 0.50764 as the 512^3 vortex
at Re = 1600, so the same per-step dissipation at the grid scale) with FP64,
FP32, FP16 (nearest and stochastic rounding) and BF16 (stochastic rounding)
populations advanced together for 1000 steps, every step through the fused
reductions (cmlbm_step_reduce) so that each run's kinetic energy is known at
every step.

Bars:
- the FP64 run itself within 1e-12 (relative L2 velocity, eq. error) of the
  80-bit oracle after the 1000 steps, so the FP64 run is a valid judge;
- FP32 within 1e-5 of the FP64 run at every checkpoint;
- FP16 with stochastic rounding within 1e-3 of the FP64 run at every
  checkpoint (the precision target for 16-bit storage), and its kinetic
  energy within 1e-3 of the FP64 run's at every step.
FP16 with nearest rounding and BF16 are reported, not bounded here.
"""
import io
import json
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

N, RE, STEPS, EVERY = 64, 200.0, 1000, 250


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_lockstep_taylor_green_64():
    import torch
    from paper_1905_10182_amd import studies

    log(f"lockstep TGV {N}^3 Re {RE}: fp64 fp32 fp16 fp16sr bf16sr, {STEPS} steps")
    wl = W.taylor_green(N, re=RE, seed=1)
    lats = {}
    for st in ("fp64", "fp32", "fp16", "fp16sr", "bf16sr"):
        lats[st] = studies._make(st, N, wl["tau"], fused=True)
        lats[st].init(wl["rho"], wl["u"])
    buf = io.StringIO()
    ke = []
    rows = studies.lockstep(lats, STEPS, EVERY, f"taylor_green_{N}_re{int(RE)}", out=buf, per_step_ke=True,
                            ke_rows=ke)
    for r in rows:
        log("  " + json.dumps({k: (round(v, 9) if isinstance(v, float) else v) for k, v in r.items()
                               if k.startswith("err_") and k.endswith("vs_fp64") or k == "step"}))
    assert [r["step"] for r in rows] == list(range(0, STEPS + 1, EVERY))
    assert len(ke) == STEPS
    for r in rows:
        assert r["err_fp32_vs_fp64"] < 1e-5, r
        assert r["err_fp16sr_vs_fp64"] < 1e-3, r
        assert all(np.isfinite(v) for k, v in r.items() if k.startswith("err_"))
    dke = max(abs(k["fp16sr"] / k["fp64"] - 1) for k in ke)
    dke32 = max(abs(k["fp32"] / k["fp64"] - 1) for k in ke)
    log(f"  max relative kinetic-energy deviation from fp64 over {STEPS} steps: fp16sr {dke:.3e}, fp32 {dke32:.3e}")
    assert dke < 1e-3 and dke32 < 1e-5
    # the judge itself: the FP64 run against the 80-bit oracle
    ref = O.Lattice(N, N, N, tau=wl["tau"], extended=True)
    ref.init(wl["rho"], wl["u"])
    ref.step(STEPS)
    _, ur = ref.moments()
    ur = np.asarray(ur, np.float64)
    u = lats["fp64"].moments()[1].cpu().numpy()
    err = float(np.linalg.norm(u - ur) / np.linalg.norm(ur))
    log(f"  fp64 run vs 80-bit oracle after {STEPS} steps: {err:.3e}")
    assert err < 1e-12
    for lat in lats.values():
        lat.close()
    torch.cuda.synchronize()
