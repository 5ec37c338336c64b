"""Parity of the HIP magnetic lattice and the Lorentz-force coupling
(include/cmlbm_mhd.h with the fluid of include/cmlbm.h) against the CPU
oracle (oracle/mhd_oracle.c with the D3Q27 oracle).

Tolerances: FP64 1e-12 relative against the 80-bit oracle; FP32 1e-5
relative.
"""
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import mhd as M

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


SHAPES = [(37, 5, 3), (64, 16, 1), (1, 1, 1), (5, 1, 7)]


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
@pytest.mark.parametrize("nx,ny,nz", SHAPES)
def test_magnetic_steps_and_fields_match_oracle(torch, storage, nx, ny, nz):
    from paper_1905_10182_amd.mhd import MagneticLattice

    log(f"mhd {storage} {nx}x{ny}x{nz}: 6 steps with a velocity field, then b, j, F")
    g = W.generator(nx * 7 + ny * 3 + nz)
    shape = (nz, ny, nx)
    b = g.uniform(-0.05, 0.05, (3,) + shape)
    u = g.uniform(-0.05, 0.05, (3,) + shape)
    ref = M.MagneticLattice(nx, ny, nz, 0.7, extended=storage == "fp64")
    ref.init(b, u)
    ref.h += np.asarray(g.uniform(-1e-3, 1e-3, ref.h.shape), ref.h.dtype)  # off equilibrium
    lat = MagneticLattice(nx, ny, nz, 0.7, storage=storage, device="cuda:0")
    lat.load_populations(np.asarray(ref.h, np.float64))
    for _ in range(6):
        ref.step(u)
        lat.step(u)
    assert lat.time == 6
    hp = lat.populations().cpu().numpy()
    tol = 1e-12 if storage == "fp64" else 1e-5
    assert rel(hp, ref.h) < tol
    for current in ("populations", "stencil"):
        ut = torch.as_tensor(u, dtype=lat.dtype, device="cuda:0")
        F = torch.empty((3,) + shape, dtype=lat.dtype, device="cuda:0")
        bg, jg = lat.fields(ut, current, F_out=F)
        br, jr = ref.fields(u, current)
        Fr = M.lorentz(np.asarray(jr, np.float64), np.asarray(br, np.float64))
        assert rel(bg.cpu().numpy(), br) < tol
        if np.linalg.norm(np.asarray(jr, np.float64)) > 0:
            assert rel(jg.cpu().numpy(), jr) < (1e-11 if storage == "fp64" else 1e-4), current
            assert rel(F.cpu().numpy(), Fr) < (1e-11 if storage == "fp64" else 1e-4), current
        else:  # one cell: the curl of a constant field is zero
            assert abs(jg.cpu().numpy()).max() < 1e-12


def orszag_tang(n, Ma):
    """Two-dimensional Orszag-Tang fields on an n x n x 1 box: u = u0 (-sin y,
    sin x), b = u0 (-sin y, sin 2x) with u0 = Ma cs, node coordinates scaled
    to a 2 pi box."""
    u0 = Ma / math.sqrt(3.0)
    k = 2 * math.pi / n
    X, Y = np.meshgrid(np.arange(n), np.arange(n))
    u = np.zeros((3, 1, n, n))
    b = np.zeros((3, 1, n, n))
    u[0, 0] = -u0 * np.sin(k * Y)
    u[1, 0] = u0 * np.sin(k * X)
    b[0, 0] = -u0 * np.sin(k * Y)
    b[1, 0] = u0 * np.sin(2 * k * X)
    return u, b


@pytest.mark.parametrize("storage,model,current", [("fp64", "m1", "populations"), ("fp64", "m5", "stencil"),
                                                   ("fp32", "m1", "populations")])
def test_coupled_orszag_tang_matches_oracle(torch, storage, model, current):
    from paper_1905_10182_amd.mhd import CoupledMHD

    n, steps = 32, 100
    log(f"coupled MHD {storage} {model} {current}: Orszag-Tang {n}^2, {steps} steps")
    u, b = orszag_tang(n, 0.14)
    tau, tau_m = 0.52, 0.53
    ref = M.MHD(n, n, 1, tau, tau_m, variant="closed" if model == "m1" else model, current=current,
                extended=storage == "fp64")
    ref.init(np.ones((1, n, n)), u, b)
    ref.step(steps)
    rr, ur, br, jr = ref.state()
    S = CoupledMHD(n, n, 1, tau, tau_m, storage=storage, model=model, current=current)
    S.init(np.ones((1, n, n)), u, b)
    S.step(steps)
    assert S.time == steps
    rg, ug, bg, jg = (t.cpu().numpy() for t in S.state())
    tol = 1e-12 if storage == "fp64" else 1e-5
    assert rel(ug, ur) < tol and rel(bg, br) < tol
    assert rel(jg, jr) < 10 * tol
    assert abs(rg - np.asarray(rr, np.float64)).max() < tol


def test_alfven_wave_on_gpu(torch):
    """The coupled GPU solver reproduces the Alfven frequency k B0 (stencil
    current) to the accuracy the oracle shows at this resolution."""
    from paper_1905_10182_amd.mhd import CoupledMHD

    n, B0, eps, tau = 64, 0.05, 1e-4, 0.6
    k = 2 * math.pi / n
    x = np.arange(n)
    b = np.zeros((3, 1, 1, n))
    b[0] = B0
    b[1, 0, 0] = eps * np.cos(k * x)
    S = CoupledMHD(n, 1, 1, tau, tau, storage="fp64", current="stencil")
    S.init(np.ones((1, 1, n)), np.zeros((3, 1, 1, n)), b)
    nu, eta = (tau - 0.5) / 3, (tau - 0.5) / 4
    w = math.sqrt(k * k * B0 * B0 - ((nu - eta) * k * k / 2) ** 2)
    c = torch.as_tensor(np.cos(k * x), device="cuda:0")
    ser = []
    for _ in range(int(2.2 * math.pi / w)):
        ser.append(float(S.mag.fields()[0][1, 0, 0] @ c))
        S.step()
    z = [i + ser[i] / (ser[i] - ser[i + 1]) for i in range(len(ser) - 1) if ser[i] * ser[i + 1] < 0]
    err = math.pi / (z[1] - z[0]) / w - 1
    log(f"  Alfven frequency error at n = {n}: {err:.3e}")
    assert abs(err) < 2e-3
