"""The FP64 global monitors of the GPU path -- cmlbm_reduce and the fused
cmlbm_step_reduce -- against the oracle's reductions of the same state
(oracle.reductions on the oracle's own moments, eq. macroscopic): mass,
momentum sum_i f_i c_i, kinetic energy sum rho |u|^2 / 2 with the
half-force-corrected u, max |u|, sum |u|^2, the residual between two states
(sum |u - u_snapshot|^2 and its relative L2 norm, eq. error), and the fluid
and non-finite counts.

State: a ragged batch of two lattices (70 or 37 cells per row), halfway
bounce-back walls on y and z, solid nodes, a per-cell force field, and
random non-equilibrium populations f = w (1 + eps), eps ~ U(-0.2, 0.2).  The
shifted values f - w and the force are chosen on the host so that the
storage format holds them exactly; both sides start from these same numbers
(no input comes from the GPU).

Bars:
- cmlbm_reduce forms every per-cell value in FP64 from the stored numbers, for
  every storage type: 1e-12 relative against the oracle (80-bit build for
  FP64 storage, FP64 build otherwise).
- cmlbm_step_reduce forms the per-cell values with the step's own arithmetic,
  FP64 for FP64 storage (1e-12) and FP32 otherwise: per cell |du| <= ~1e-8
  here (|u| ~ 0.04, 27 terms of |f - w| <= 0.2 w rounded at 2^-24), so the
  energy-type sums agree to 2e-6 relative, max |u| to 2e-6, and the mass and
  momentum sums to 1e-7 per fluid cell.
"""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

CX, CY, CZ, WGT, OPP = O.constants()
RED = {"mass": 0, "momx": 1, "momy": 2, "momz": 3, "ke": 4, "umax": 5, "nonfinite": 6, "fluid": 7,
       "du2": 8, "u2": 9, "residual": 10}
NY, NZ, NB = 13, 9, 2
TAU = 0.73


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def make_state(storage, nx, seed, solid):
    """Populations (27, nb, nz, ny, nx) whose shifted values the format holds
    exactly; solid cells hold zeros (never read)."""
    shape = (NB, NZ, NY, nx)
    g = W.generator(seed)
    w = WGT.reshape((27, 1, 1, 1, 1))
    h = W.representable(w * g.uniform(-0.2, 0.2, size=(27,) + shape), storage)
    f = w + h
    f[:, solid.astype(bool)] = 0.0
    return f


def geometry(storage, nx, seed=101):
    shape = (NB, NZ, NY, nx)
    g = W.generator(seed)
    solid = (g.uniform(size=shape) < 0.08).astype(np.uint8)
    force = W.representable(g.uniform(-1e-3, 1e-3, size=(3,) + shape), "fp64" if storage == "fp64" else "fp32")
    return solid, force


def oracle_lattice(storage, nx, solid, force):
    return O.Lattice(nx, NY, NZ, nb=NB, tau=TAU, wall=(0, 1, 1), solid=solid, force=force,
                     extended=storage == "fp64")


def gpu_lattice(storage, nx, solid, force):
    from paper_1905_10182_amd import Lattice
    lat = Lattice(nx, NY, NZ, nbatch=NB, tau=TAU, storage=storage, wall=(0, 1, 1), solid=True, residual=True,
                  fused_reduce=True, device="cuda:0")
    lat.set_solid(solid)
    lat.set_force("field", field=force)
    return lat


def compare(got, ref, rtol_sum, atol_cell, rtol_max, label):
    """got: (nb, NRED) from the GPU; ref: the oracle's per-member dicts."""
    for b, d in enumerate(ref):
        n = d["fluid"]
        assert got[b, RED["fluid"]] == n, (label, b)
        assert got[b, RED["nonfinite"]] == d["nonfinite"], (label, b)
        if d["nonfinite"]:
            continue
        np.testing.assert_allclose(got[b, RED["mass"]], float(d["mass"]), rtol=0, atol=atol_cell * n,
                                   err_msg=f"{label} mass {b}")
        np.testing.assert_allclose(got[b, 1:4], np.asarray(d["mom"], np.float64), rtol=0, atol=atol_cell * n,
                                   err_msg=f"{label} momentum {b}")
        for key in ("ke", "u2"):
            np.testing.assert_allclose(got[b, RED[key]], float(d[key]), rtol=rtol_sum, atol=0,
                                       err_msg=f"{label} {key} {b}")
        np.testing.assert_allclose(got[b, RED["umax"]], float(d["umax"]), rtol=rtol_max, atol=0,
                                   err_msg=f"{label} umax {b}")
        log(f"  {label} member {b}: ke {got[b, RED['ke']]:.12e} oracle {float(d['ke']):.12e}, "
            f"umax {got[b, RED['umax']]:.9e} oracle {float(d['umax']):.9e}")


# relative bars of the residual after two steps: the GPU state after a step
# is the oracle's up to the step's FP64 / FP32 arithmetic and the rounding of
# the stored format (half a unit of FP16's 11-bit / BF16's 8-bit significand
# on |f - w|), relative to a two-step change |u_t - u_{t-2}| ~ |u|
RESIDUAL_RTOL = {"fp64": 1e-12, "fp32": 1e-5, "fp16": 2e-3, "bf16": 2e-2}


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16", "bf16"])
@pytest.mark.parametrize("nx", [70, 37])
def test_reduce_and_residual_match_oracle(torch, storage, nx):
    """cmlbm_reduce of a loaded state (every sum, 1e-12), and the residual
    between that state (the snapshot) and the state two steps later."""
    log(f"{storage} cmlbm_reduce vs oracle, {nx}x{NY}x{NZ} x{NB}, walls y z, solids, field force")
    solid, force = geometry(storage, nx)
    fa = make_state(storage, nx, 7, solid)
    ref = oracle_lattice(storage, nx, solid, force)
    ref.load_populations(fa)
    ra = ref.reductions()
    ua = ref.moments()[1]
    ref.step(2)
    rb = ref.reductions(u_snapshot=ua)
    lat = gpu_lattice(storage, nx, solid, force)
    lat.load_populations(fa)
    got_a = lat.reduce(snapshot=True)
    compare(got_a, ra, 1e-12, 1e-13, 1e-12, "state a")
    assert np.all(got_a[:, RED["du2"]] == 0) and np.all(got_a[:, RED["residual"]] == 0)
    assert np.array_equal(got_a, lat.reduce())  # fixed summation order
    lat.step(2)
    got_b = lat.reduce(residual=True)
    tol = RESIDUAL_RTOL[storage]
    for b, d in enumerate(rb):
        log(f"  residual member {b}: {got_b[b, RED['residual']]:.12e} oracle {float(d['residual']):.12e}")
        np.testing.assert_allclose(got_b[b, RED["du2"]], float(d["du2"]), rtol=tol, atol=0)
        np.testing.assert_allclose(got_b[b, RED["residual"]], float(d["residual"]), rtol=tol, atol=0)
        assert 0.05 < float(d["residual"]) < 20  # a change the bars above resolve
    lat.close()


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16", "bf16"])
@pytest.mark.parametrize("nx", [70, 37])
def test_step_reduce_matches_oracle(torch, storage, nx):
    """The fused kernel's sums of the state it reads (time t), then the
    next call's sums of the state the step wrote (time t + 1) against the
    oracle stepped once from the same state."""
    log(f"{storage} cmlbm_step_reduce vs oracle, {nx}x{NY}x{NZ} x{NB}, walls y z, solids, field force")
    solid, force = geometry(storage, nx)
    fa = make_state(storage, nx, 7, solid)
    ref = oracle_lattice(storage, nx, solid, force)
    ref.load_populations(fa)
    r0 = ref.reductions()
    ref.step(1)
    r1 = ref.reductions()
    lat = gpu_lattice(storage, nx, solid, force)
    lat.load_populations(fa)
    if storage == "fp64":
        tol = dict(rtol_sum=1e-12, atol_cell=1e-13, rtol_max=1e-12)
    else:
        tol = dict(rtol_sum=2e-6, atol_cell=1e-7, rtol_max=2e-6)
    compare(lat.step_reduce(), r0, label="t", **tol)
    if storage in ("fp16", "bf16"):
        # the state at t + 1 is the 16-bit rounding of the step's output: each
        # population is off by up to half a unit of the format, so the sums
        # agree to that rounding (2^-12 of |f - w| for FP16, 2^-9 for BF16)
        tol = dict(rtol_sum=5e-3 if storage == "bf16" else 5e-4, atol_cell=1e-4, rtol_max=5e-3)
    compare(lat.step_reduce(), r1, label="t+1", **tol)
    assert lat.time == 2
    lat.close()


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16"])
def test_members_are_reduced_apart(torch, storage):
    """A non-finite population in member 1 is counted there (EUNSTABLE), and
    member 0's sums still match the oracle, through both entry points."""
    nx = 70
    log(f"{storage} non-finite cell in member 1 only")
    solid, force = geometry(storage, nx)
    f = make_state(storage, nx, 9, solid)
    fl = np.argwhere(solid[1] == 0)[17]
    f[4, 1, fl[0], fl[1], fl[2]] = np.nan
    ref = oracle_lattice(storage, nx, solid, force)
    ref.load_populations(f)
    rr = ref.reductions()
    assert rr[1]["nonfinite"] == 1 and rr[0]["nonfinite"] == 0
    lat = gpu_lattice(storage, nx, solid, force)
    lat.load_populations(f)
    tol = 1e-12 if storage == "fp64" else 2e-6
    got = lat.reduce(allow_unstable=True)
    compare(got, rr, 1e-12, 1e-13, 1e-12, "reduce")
    got = lat.step_reduce(allow_unstable=True)
    compare(got, rr, tol, 1e-13 if storage == "fp64" else 1e-7, tol, "step_reduce")
    lat.close()


def oracle_blow_up_step(n=32, u0=0.3, tau=0.5005, every=5, limit=400):
    """First multiple of `every` at which the oracle's state has a non-finite
    cell (the unstable Taylor-Green run of the oracle's blow-up test)."""
    wl = W.taylor_green(n, seed=1, u0=u0)
    ref = O.Lattice(n, n, n, tau=tau)
    ref.init(wl["rho"], wl["u"])
    for k in range(every, limit + 1, every):
        ref.step(every)
        with np.errstate(invalid="ignore", over="ignore"):
            if ref.reductions()[0]["nonfinite"]:
                return k
    return None


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_blow_up_reports_unstable(torch, storage):
    """The unstable run (TGV 32^3, u0 = 0.3, tau = 0.5005) through the
    library: cmlbm_reduce raises EUNSTABLE once the state turns non-finite
    and not before (both sides checked every 5 steps); in FP64 it fires
    within 20 steps of the oracle's detector."""
    from paper_1905_10182_amd import Lattice
    from paper_1905_10182_amd import cmlbm as B
    k_ref = oracle_blow_up_step()
    assert k_ref is not None
    log(f"{storage} blow-up run, TGV 32^3 u0 = 0.3 tau = 0.5005; oracle fires at step {k_ref}")
    wl = W.taylor_green(32, seed=1, u0=0.3)
    lat = Lattice(32, 32, 32, tau=0.5005, storage=storage, device="cuda:0")
    lat.init(wl["rho"], wl["u"])
    fired = None
    for k in range(5, 401, 5):
        lat.step(5)
        try:
            r = lat.reduce()
        except B.CmlbmError as e:
            assert e.code == B.EUNSTABLE
            fired = k
            break
        assert np.isfinite(r[0, RED["ke"]]) and r[0, RED["nonfinite"]] == 0
    log(f"  library fires at step {fired}")
    assert fired is not None
    r = lat.reduce(allow_unstable=True)
    assert r[0, RED["nonfinite"]] > 0 and r[0, RED["fluid"]] == 32 ** 3
    if storage == "fp64":
        assert abs(fired - k_ref) <= 20
    lat.close()
