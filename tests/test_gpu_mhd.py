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


# ---------------------------------------------------------------------------
# walls and the Hartmann flow

@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_magnetic_walls_match_oracle(torch, storage):
    from paper_1905_10182_amd.mhd import MagneticLattice

    nx, ny, nz = 13, 6, 4
    log(f"mhd walls {storage} {nx}x{ny}x{nz}, walls on y and z")
    g = W.generator(41)
    shape = (nz, ny, nx)
    bw = np.array([0.01, 0.03, -0.02])
    b = g.uniform(-0.05, 0.05, (3,) + shape)
    u = g.uniform(-0.05, 0.05, (3,) + shape)
    ref = M.MagneticLattice(nx, ny, nz, 0.7, extended=storage == "fp64", wall=(0, 1, 1), b_wall=bw)
    ref.init(b, u)
    ref.h += np.asarray(g.uniform(-1e-3, 1e-3, ref.h.shape), ref.h.dtype)
    lat = MagneticLattice(nx, ny, nz, 0.7, storage=storage, device="cuda:0", wall=(0, 1, 1), b_wall=bw)
    lat.load_populations(np.asarray(ref.h, np.float64))
    tol = 1e-12 if storage == "fp64" else 1e-5
    assert rel(lat.populations().cpu().numpy(), ref.h) < tol  # the wall-aware scatter inverts the gather
    for _ in range(6):
        ref.step(u)
        lat.step(u)
    assert rel(lat.populations().cpu().numpy(), ref.h) < tol
    for current in ("populations", "stencil"):
        bg, jg = lat.fields(torch.as_tensor(u, dtype=lat.dtype, device="cuda:0"), current)
        br, jr = ref.fields(u, current)
        assert rel(bg.cpu().numpy(), br) < tol
        assert rel(jg.cpu().numpy(), jr) < (1e-11 if storage == "fp64" else 1e-4), current


def hartmann_setup(L, Ha, nu=0.1, umax=1e-3):
    a = L / 2.0
    B0 = Ha * nu / a
    G = umax * nu * Ha * math.tanh(Ha) / (a * a)
    s = np.arange(L) - (L - 1) / 2.0
    ua = G * a * a / (nu * Ha * math.tanh(Ha)) * (1 - np.cosh(Ha * s / a) / math.cosh(Ha))
    return a, B0, G, ua


def test_coupled_hartmann_matches_oracle(torch):
    from paper_1905_10182_amd.mhd import CoupledMHD

    L, Ha, nu, steps = 24, 5.0, 0.1, 400
    log(f"coupled Hartmann L={L} Ha={Ha}: {steps} steps against the 80-bit oracle")
    a, B0, G, _ = hartmann_setup(L, Ha, nu)
    b = np.zeros((3, 1, L, 1))
    b[1] = B0
    ref = M.MHD(1, L, 1, 0.5 + 3 * nu, 0.5 + 4 * nu, current="populations", extended=True, wall=(0, 1, 0),
                b_wall=(0.0, B0, 0.0))
    ref.init(np.ones((1, L, 1)), np.zeros((3, 1, L, 1)), b)
    ref.body_force = (G, 0.0, 0.0)
    ref.step(steps)
    _, ur, br, _ = ref.state()
    S = CoupledMHD(1, L, 1, 0.5 + 3 * nu, 0.5 + 4 * nu, storage="fp64", current="populations", wall=(0, 1, 0),
                   b_wall=(0.0, B0, 0.0), body_force=(G, 0.0, 0.0))
    S.init(np.ones((1, L, 1)), np.zeros((3, 1, L, 1)), b)
    S.step(steps)
    _, ug, bg, _ = (t.cpu().numpy() for t in S.state())
    assert rel(ug, ur) < 1e-12 and rel(bg, br) < 1e-12


def test_hartmann_steady_profile_on_gpu(torch):
    """The coupled GPU solver reaches the analytic Hartmann profile: at
    Ha = 10 the error falls at second order from L = 32 to 64."""
    from paper_1905_10182_amd.mhd import CoupledMHD

    nu, Ha, errs = 0.1, 10.0, []
    for L in (32, 64):
        a, B0, G, ua = hartmann_setup(L, Ha, nu)
        b = np.zeros((3, 1, L, 1))
        b[1] = B0
        S = CoupledMHD(1, L, 1, 0.5 + 3 * nu, 0.5 + 4 * nu, storage="fp64", current="populations", wall=(0, 1, 0),
                       b_wall=(0.0, B0, 0.0), body_force=(G, 0.0, 0.0))
        S.init(np.ones((1, L, 1)), np.zeros((3, 1, L, 1)), b)
        S.step(int(48 * a * a / (nu * (math.pi ** 2 + Ha ** 2))) + 200)
        u = S.state()[1][0, 0, :, 0].cpu().numpy()
        errs.append(rel(u, ua))
        log(f"  L={L}: error {errs[-1]:.3e}")
    assert errs[1] < 6e-3 and math.log2(errs[0] / errs[1]) > 1.8, errs


def test_bench_size_magnetic_step_sampled(torch):
    """The magnetic lattice in the benchmark's configuration (256^3, FP32,
    periodic, a fixed velocity field, 256-thread workgroups): one step on 2048
    sampled cells against the oracle's collision (App. C equilibrium) of the
    exported populations at x - xi_l, streamed to x."""
    from paper_1905_10182_amd.mhd import MagneticLattice
    n, tau_m = 256, 0.8
    log(f"magnetic lattice {n}^3 fp32, one step, 2048 sampled cells")
    lat = MagneticLattice(n, n, n, tau_m, storage="fp32", device="cuda:0")
    c = torch.arange(n, device="cuda:0", dtype=torch.float32) * (2 * math.pi / n)
    z, y, x = torch.meshgrid(c, c, c, indexing="ij")
    b = torch.stack([torch.sin(y), torch.sin(z), torch.sin(x)]) * 0.01
    u = (torch.stack([torch.sin(z), torch.sin(x), torch.sin(y)]) * 0.02).contiguous()
    lat.init(b, u)
    lat.step(u)  # leave equilibrium
    del b, x, y, z
    xi, _ = M.constants()
    g = W.generator(41)
    s = np.stack([g.integers(0, n, 2048), g.integers(0, n, 2048), g.integers(0, n, 2048)], 1)  # (x, y, z)
    lin = lambda q: torch.as_tensor((q[:, 2] * n + q[:, 1]) * n + q[:, 0], device="cuda:0")
    P0 = lat.populations().reshape(7, 3, -1)
    src = {l: (s - xi[l]) % n for l in range(7)}
    h0 = {l: P0[:, :, lin(src[l])].cpu().numpy() for l in range(7)}  # (7, 3, 2048) at x - xi_l
    u0 = {l: u.reshape(3, -1)[:, lin(src[l])].double().cpu().numpy() for l in range(7)}
    del P0
    lat.step(u)
    P1 = lat.populations().reshape(7, 3, -1)[:, :, lin(s)].cpu().numpy()
    om = 1.0 / tau_m
    err = 0.0
    for l in range(7):
        for k in range(len(s)):
            hp = h0[l][:, :, k]
            e = M.heq(hp.sum(axis=0), u0[l][:, k])
            want = hp[l] + om * (e[l] - hp[l])
            err = max(err, float(np.abs(P1[l, :, k] - want).max()))
    log(f"  max |h - oracle| = {err:.3e}")
    assert err < 2e-9  # FP32 arithmetic on populations of order 1e-3


def test_planes_over_2gib_magnetic_step_sampled(torch):
    """The magnetic lattice with population planes of 2.03 GiB (1024 x 1024 x
    520, FP32: in-plane byte offsets past 2^31), from a seeded per-cell random
    field b (components within +-0.01) and velocity u (within +-0.02) drawn on
    the device: one step on 2056 sampled cells (the corners among them) against
    the oracle's collision of the exported populations at x - xi_l."""
    from paper_1905_10182_amd.mhd import MagneticLattice
    nx, ny, nz, tau_m = 1024, 1024, 520, 0.8
    n = nx * ny * nz
    need = 2 * 21 * 4 * n + 21 * 8 * n + 24 * n + (2 << 30)
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory, {free / 2**30:.0f} GiB free")
    log(f"magnetic lattice {nx}x{ny}x{nz} fp32: {21 * 4 * n / 2**30:.0f} GiB of populations per buffer")
    lat = MagneticLattice(nx, ny, nz, tau_m, storage="fp32", device="cuda:0")
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(520)
    b = 0.02 * (torch.rand((3, nz, ny, nx), generator=gen, device="cuda:0") - 0.5)
    u = 0.04 * (torch.rand((3, nz, ny, nx), generator=gen, device="cuda:0") - 0.5)
    lat.init(b, u)
    del b
    torch.cuda.empty_cache()
    xi, _ = M.constants()
    g = W.generator(520)
    corners = np.array([[x, y, z] for x in (0, nx - 1) for y in (0, ny - 1) for z in (0, nz - 1)])
    s = np.concatenate([corners, np.stack([g.integers(0, nx, 2048), g.integers(0, ny, 2048),
                                           g.integers(0, nz, 2048)], 1)])  # (x, y, z)
    dims3 = np.array([nx, ny, nz])
    lin = lambda q: torch.as_tensor((q[:, 2] * ny + q[:, 1]) * nx + q[:, 0], device="cuda:0")
    P0 = lat.populations().reshape(7, 3, -1)
    src = {l: (s - xi[l]) % dims3 for l in range(7)}
    h0 = {l: P0[:, :, lin(src[l])].cpu().numpy() for l in range(7)}  # (7, 3, n) at x - xi_l
    u0 = {l: u.reshape(3, -1)[:, lin(src[l])].double().cpu().numpy() for l in range(7)}
    del P0
    torch.cuda.empty_cache()
    lat.step(u)
    P1 = lat.populations().reshape(7, 3, -1)[:, :, lin(s)].cpu().numpy()
    lat.close()
    del lat, u
    torch.cuda.empty_cache()
    om = 1.0 / tau_m
    err = 0.0
    for l in range(7):
        for k in range(len(s)):
            hp = h0[l][:, :, k]
            e = M.heq(hp.sum(axis=0), u0[l][:, k])
            want = hp[l] + om * (e[l] - hp[l])
            err = max(err, float(np.abs(P1[l, :, k] - want).max()))
    log(f"  max |h - oracle| = {err:.3e}")
    assert err < 2e-9
