"""Parity of the HIP solver (through the C ABI) with the CPU oracle.

Tolerances: FP64 storage 1e-12 relative, FP32 storage 1e-5 relative in
velocity (relative L2 over fluid cells), 16-bit storage checked per
population against round-to-nearest of the oracle's post-collision value.

FP64-storage runs are compared with the oracle built in 80-bit long double:
on slow flows (Poiseuille, |u| ~ 3e-4) the FP64 textbook form's own rounding
of sum f c over populations of order 1 is about 2e-12 relative in u, above
the 1e-12 bar, while the extended build is exact to that bar.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

CX, CY, CZ, WGT, OPP = O.constants()


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def Lat(**kw):
    from paper_1905_10182_amd import Lattice
    return Lattice(device="cuda:0", **kw)


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def fluid_rel(u, ref, solid=None):
    if solid is None:
        return rel(u, ref)
    m = ~np.asarray(solid, bool)
    return rel(np.asarray(u)[:, m], np.asarray(ref)[:, m])


def tgv_pair(n, storage, steps, re=1600.0, stochastic=False):
    wl = W.taylor_green(n, re=re, seed=1)
    ref = O.Lattice(n, n, n, tau=wl["tau"], extended=storage == "fp64")
    ref.init(wl["rho"], wl["u"])
    ref.step(steps)
    lat = Lat(nx=n, ny=n, nz=n, tau=wl["tau"], storage=storage, stochastic=stochastic)
    lat.init(wl["rho"], wl["u"])
    lat.step(steps)
    return ref, lat


# ---------------------------------------------------------------------------
# state import/export

def test_population_roundtrip_bit_exact_fp64(torch):
    """load_populations followed by populations is the identity (the init
    scatter is the exact inverse of the pull gather) on a ragged batch with
    walls on two axes and solid nodes."""
    log("roundtrip fp64 37x13x11 nb=2")
    shape = (2, 11, 13, 37)
    g = W.generator(21)
    solid = (g.uniform(size=shape) < 0.1).astype(np.uint8)
    f = WGT.reshape(27, 1, 1, 1, 1) * g.uniform(0.6, 1.6, size=(27,) + shape)  # f in [w/2, 2w]
    f[:, solid.astype(bool)] = 0.0
    lat = Lat(nx=37, ny=13, nz=11, nbatch=2, tau=0.7, storage="fp64", wall=(0, 1, 1), solid=True)
    lat.set_solid(solid)
    lat.load_populations(f)
    out = lat.populations().cpu().numpy()
    assert np.array_equal(out, f)


def test_population_roundtrip_fp32(torch):
    log("roundtrip fp32 40x9x7")
    shape = (1, 7, 9, 40)
    f = WGT.reshape(27, 1, 1, 1, 1) * W.generator(22).uniform(0.6, 1.6, size=(27,) + shape)
    lat = Lat(nx=40, ny=9, nz=7, tau=0.7, storage="fp32")
    lat.load_populations(f)
    out = lat.populations().cpu().numpy()
    dev = (f - WGT.reshape(27, 1, 1, 1, 1)).astype(np.float32).astype(np.float64) + WGT.reshape(27, 1, 1, 1, 1)
    np.testing.assert_array_equal(out, dev)


# ---------------------------------------------------------------------------
# FP64 parity

def test_fp64_random_state_field_force_walls_solid(torch):
    """Non-equilibrium random populations, per-cell force field, walls in y
    and z, solid nodes, a ragged batch of two: 5 steps, every population."""
    log("fp64 random state 37x13x11 nb=2, 5 steps")
    shape = (2, 11, 13, 37)
    g = W.generator(23)
    solid = (g.uniform(size=shape) < 0.08).astype(np.uint8)
    f0 = W.random_populations(shape, seed=24)
    f0[:, solid.astype(bool)] = 0.0
    force = g.uniform(-1e-3, 1e-3, size=(3,) + shape)
    ref = O.Lattice(37, 13, 11, nb=2, tau=0.73, wall=(0, 1, 1), solid=solid, force=force, extended=True)
    ref.load_populations(f0)
    ref.step(5)
    lat = Lat(nx=37, ny=13, nz=11, nbatch=2, tau=0.73, storage="fp64", wall=(0, 1, 1), solid=True)
    lat.set_solid(solid)
    lat.set_force("field", field=force)
    lat.load_populations(f0)
    lat.step(5)
    out = lat.populations().cpu().numpy()
    fr = ref.f.astype(np.float64)
    err = np.abs(out - fr).max() / np.abs(fr).max()
    log(f"  max population error {err:.3e}")
    assert err < 1e-13
    rho, u = lat.moments()
    rr, ur = ref.moments()
    assert fluid_rel(u.cpu().numpy(), ur, solid) < 1e-12
    m = ~solid.astype(bool)
    assert rel(rho.cpu().numpy()[m], rr[m]) < 1e-14


def test_fp64_taylor_green_32(torch):
    log("fp64 TGV 32^3, 200 steps")
    ref, lat = tgv_pair(32, "fp64", 200)
    _, u = lat.moments()
    _, ur = ref.moments()
    err = rel(u.cpu().numpy(), ur)
    perr = rel(lat.populations().cpu().numpy(), ref.f)
    log(f"  velocity {err:.3e} populations {perr:.3e}")
    assert err < 1e-12 and perr < 1e-12


def test_fp64_poiseuille_config(torch):
    """Body-force Poiseuille channel 32x16x16, tau 0.8, F_x 1e-6, 1000 steps."""
    log("fp64 Poiseuille 32x16x16, 1000 steps")
    wl = W.poiseuille()
    nb, nz, ny, nx = wl["shape"]
    ref = O.Lattice(nx, ny, nz, tau=wl["tau"], wall=wl["wall"], force=wl["force"].reshape(3, 1, 1, 1, 1),
                    extended=True)
    ref.init(wl["rho"], wl["u"])
    ref.step(wl["steps"])
    lat = Lat(nx=nx, ny=ny, nz=nz, tau=wl["tau"], storage="fp64", wall=wl["wall"])
    lat.set_force("uniform", wl["force"])
    lat.init(wl["rho"], wl["u"])
    lat.step(wl["steps"])
    _, u = lat.moments()
    _, ur = ref.moments()
    err = rel(u.cpu().numpy(), ur)
    log(f"  velocity {err:.3e}")
    assert err < 1e-12


def test_fp64_kolmogorov_profile_force(torch):
    log("fp64 Kolmogorov 48^3, 100 steps")
    wl = W.kolmogorov(48, f0=1e-4, tau=0.6)
    prof = wl["force_profile_y"]
    field = np.broadcast_to(prof.T[:, None, None, :, None], (3,) + wl["shape"])
    ref = O.Lattice(48, 48, 48, tau=wl["tau"], force=field, extended=True)
    ref.init(wl["rho"], wl["u"])
    ref.step(100)
    lat = Lat(nx=48, ny=48, nz=48, tau=wl["tau"], storage="fp64")
    lat.set_force("profile_y", prof)
    lat.init(wl["rho"], wl["u"])
    lat.step(100)
    _, u = lat.moments()
    _, ur = ref.moments()
    err = rel(u.cpu().numpy(), ur)
    log(f"  velocity {err:.3e}")
    assert err < 1e-12


@pytest.mark.parametrize("model", ["m4", "m5", "eq2", "bgk", "bgk6"])
def test_fp64_comparison_models_random_state(torch, model):
    """The comparison models of Sec. III (truncated equilibrium / forcing,
    same relaxation) against the oracle's literal route of the same model:
    random non-equilibrium populations, per-cell force field, walls, solids,
    a ragged batch of two, 5 steps, every population."""
    log(f"fp64 {model} random state 37x13x11 nb=2, 5 steps")
    shape = (2, 11, 13, 37)
    g = W.generator(41)
    solid = (g.uniform(size=shape) < 0.08).astype(np.uint8)
    f0 = W.random_populations(shape, seed=42)
    f0[:, solid.astype(bool)] = 0.0
    force = g.uniform(-1e-3, 1e-3, size=(3,) + shape)
    ref = O.Lattice(37, 13, 11, nb=2, tau=0.73, wall=(0, 1, 1), solid=solid, force=force, extended=True)
    ref.load_populations(f0)
    ref.step(5, variant=model)
    lat = Lat(nx=37, ny=13, nz=11, nbatch=2, tau=0.73, storage="fp64", wall=(0, 1, 1), solid=True, model=model)
    lat.set_solid(solid)
    lat.set_force("field", field=force)
    lat.load_populations(f0)
    lat.step(5)
    out = lat.populations().cpu().numpy()
    fr = ref.f.astype(np.float64)
    err = np.abs(out - fr).max() / np.abs(fr).max()
    log(f"  max population error {err:.3e}")
    assert err < 1e-13
    # and the model differs from the method on this state (the switch is live)
    m1 = O.Lattice(37, 13, 11, nb=2, tau=0.73, wall=(0, 1, 1), solid=solid, force=force)
    m1.load_populations(f0)
    m1.step(5)
    assert np.abs(out - m1.f).max() > 1e3 * err * np.abs(fr).max()


@pytest.mark.parametrize("model", ["m4", "m5"])
def test_fp32_comparison_models_taylor_green(torch, model):
    log(f"fp32 {model} TGV 32^3, 100 steps")
    wl = W.taylor_green(32, seed=1)
    ref = O.Lattice(32, 32, 32, tau=wl["tau"])
    ref.init(wl["rho"], wl["u"])
    ref.step(100, variant=model)
    lat = Lat(nx=32, ny=32, nz=32, tau=wl["tau"], storage="fp32", model=model)
    lat.init(wl["rho"], wl["u"])
    lat.step(100)
    err = rel(lat.moments()[1].cpu().numpy(), ref.moments()[1])
    log(f"  velocity {err:.3e}")
    assert err < 1e-5


# ---------------------------------------------------------------------------
# moment-representation storage (nine FP32 numbers per cell)

def test_mom32_taylor_green_32(torch):
    """Moment storage, TGV 32^3, 200 steps: within the FP32 bar of the oracle,
    and within 1e-6 of the FP32 population storage (the same arithmetic,
    streamed through on-chip memory instead of HBM)."""
    log("mom32 TGV 32^3, 200 steps")
    ref, lat32 = tgv_pair(32, "fp32", 200)
    wl = W.taylor_green(32, seed=1)
    lat = Lat(nx=32, ny=32, nz=32, tau=wl["tau"], storage="mom32")
    lat.init(wl["rho"], wl["u"])
    lat.step(200)
    u = lat.moments()[1].cpu().numpy()
    e_or = rel(u, ref.moments()[1])
    e_32 = rel(u, lat32.moments()[1].cpu().numpy())
    log(f"  vs oracle {e_or:.3e}, vs fp32 populations {e_32:.3e}")
    assert e_or < 1e-5 and e_32 < 1e-6


def test_mom32_ragged_tiles_field_force_batch(torch):
    """Partial tiles in x (70 = 64 + 6) and y (13 = 2 x 6 + 1), a partial z
    chunk (nz = 19), two batch members, a random initial field and a per-cell
    force field: 30 steps against the oracle."""
    log("mom32 70x13x19 nb=2, field force, 30 steps")
    shape = (2, 19, 13, 70)
    g = W.generator(51)
    rho0 = 1.0 + g.uniform(-1e-3, 1e-3, size=shape)
    u0 = g.uniform(-0.03, 0.03, size=(3,) + shape)
    force = g.uniform(-1e-4, 1e-4, size=(3,) + shape)
    ref = O.Lattice(70, 13, 19, nb=2, tau=0.6, force=force)
    ref.init(rho0, u0)
    ref.step(30)
    lat = Lat(nx=70, ny=13, nz=19, nbatch=2, tau=0.6, storage="mom32")
    lat.set_force("field", field=force)
    lat.init(rho0, u0)
    lat.step(30)
    rho, u = lat.moments()
    rr, ur = ref.moments()
    e_u = rel(u.cpu().numpy(), ur)
    e_r = rel(rho.cpu().numpy() - 1.0, rr - 1.0)
    log(f"  velocity {e_u:.3e} density deviation {e_r:.3e}")
    assert e_u < 1e-5 and e_r < 1e-4


def test_mom32_profile_force_and_single_plane(torch):
    """Kolmogorov profile force (48^3, 100 steps) and the four-rolls mill on a
    single z plane (16 x 16 x 1, field force, 2000 steps)."""
    log("mom32 Kolmogorov 48^3 100 steps; four-rolls 16x16x1 2000 steps")
    wl = W.kolmogorov(48, f0=1e-4, tau=0.6)
    prof = wl["force_profile_y"]
    field = np.broadcast_to(prof.T[:, None, None, :, None], (3,) + wl["shape"])
    ref = O.Lattice(48, 48, 48, tau=wl["tau"], force=field)
    ref.init(wl["rho"], wl["u"])
    ref.step(100)
    lat = Lat(nx=48, ny=48, nz=48, tau=wl["tau"], storage="mom32")
    lat.set_force("profile_y", prof)
    lat.init(wl["rho"], wl["u"])
    lat.step(100)
    e1 = rel(lat.moments()[1].cpu().numpy(), ref.moments()[1])
    # single plane: at tau = 0.50048 (omega ~ 2) and |u| ~ 1e-3 FP32 storage of
    # either kind drifts from the FP64 oracle by ~1e-4 over 2000 steps, so the
    # moment storage is held to the FP32 population storage there
    wl = W.four_rolls_mill(16)
    ref = O.Lattice(16, 16, 1, tau=wl["tau"], force=wl["force"])
    ref.init(np.ones(wl["shape"]), wl["u_exact"])
    ref.step(2000)
    out = {}
    for st in ("mom32", "fp32"):
        lat = Lat(nx=16, ny=16, nz=1, tau=wl["tau"], storage=st)
        lat.set_force("field", field=wl["force"])
        lat.init(np.ones(wl["shape"]), wl["u_exact"])
        lat.step(2000)
        out[st] = lat.moments()[1].cpu().numpy()
    e2 = rel(out["mom32"], ref.moments()[1])
    e3 = rel(out["fp32"], ref.moments()[1])
    e4 = rel(out["mom32"], out["fp32"])
    log(f"  Kolmogorov {e1:.3e}; four-rolls vs oracle: mom32 {e2:.3e} fp32 {e3:.3e}; mom32 vs fp32 {e4:.3e}")
    assert e1 < 1e-5
    assert e2 < 2 * e3 + 1e-6 and e4 < 2 * e3 + 1e-6


def test_mom32_state_semantics(torch):
    """Reductions (mass kept, momentum gains sum F per step), bitwise
    save/restore, and the refusal of population import/export."""
    from paper_1905_10182_amd.cmlbm import RED, CmlbmError, EINVAL, ESTATE
    log("mom32 reductions / checkpoint / refusals")
    # from rest the momentum gain is exactly sum F per step (in FP32 arithmetic to
    # ~1e-7; on a Taylor-Green field FP32 storage of either kind shows a ~5e-4
    # relative rounding drift of the gain, which FP64 does not)
    F = np.array([1e-6, -2e-6, 0.5e-6])
    n = 32 ** 3
    lat = Lat(nx=32, ny=32, nz=32, tau=0.6, storage="mom32")
    lat.set_force("uniform", F)
    lat.init(None, None)
    r0 = lat.reduce()[0]
    lat.step(10)
    r1 = lat.reduce()[0]
    assert abs(r1[RED["mass"]] / r0[RED["mass"]] - 1) < 1e-7
    for a, k in enumerate(("momx", "momy", "momz")):
        assert abs((r1[RED[k]] - r0[RED[k]]) / (10 * n * F[a]) - 1) < 1e-5
    wl = W.taylor_green(32, seed=1)
    lat = Lat(nx=32, ny=32, nz=32, tau=wl["tau"], storage="mom32")
    lat.set_force("uniform", F)
    lat.init(wl["rho"], wl["u"])
    r0 = lat.reduce()[0]
    lat.step(10)
    assert abs(lat.reduce()[0][RED["mass"]] / r0[RED["mass"]] - 1) < 1e-6
    blob, t = lat.save_state()
    lat.step(5)
    u5 = lat.moments()[1].clone()
    lat.restore_state(blob, t)
    lat.step(5)
    assert torch.equal(lat.moments()[1], u5)
    with pytest.raises(CmlbmError) as e:
        lat.populations()
    assert e.value.code == ESTATE
    with pytest.raises(CmlbmError) as e:
        lat.load_populations(np.zeros((27,) + lat.shape))
    assert e.value.code == EINVAL


@pytest.mark.parametrize("n", [256, 512])
def test_mom32_full_size_matches_fp32_populations(torch, n):
    """TGV 256^3 and 512^3 in the benchmark configurations: after 20 steps the
    moment storage and the FP32 population storage agree to 1e-6 in velocity
    (two independent data paths of the same arithmetic)."""
    log(f"mom32 vs fp32 populations, TGV {n}^3, 20 steps")
    wl = W.taylor_green(n, seed=1, dtype=np.float32)
    a = Lat(nx=n, ny=n, nz=n, tau=wl["tau"], storage="mom32")
    a.init(wl["rho"], wl["u"], dtype=torch.float32)
    a.step(20)
    ua = a.moments(dtype=torch.float32)[1]
    del a
    b = Lat(nx=n, ny=n, nz=n, tau=wl["tau"], storage="fp32")
    b.init(wl["rho"], wl["u"], dtype=torch.float32)
    b.step(20)
    ub = b.moments(dtype=torch.float32)[1]
    err = float(torch.linalg.vector_norm((ua - ub).double()) / torch.linalg.vector_norm(ub.double()))
    log(f"  relative difference {err:.3e}")
    assert err < 1e-6


def test_mom32_blocked_schedule_batch_field_force(torch):
    """A lattice on which the moment kernel deals its tiles to the XCDs in
    blocks of whole tile rows (256 x 96 x 40, 32 members: 4 tile columns, 8
    tile rows, two z chunks, the second of 8 planes; 8 generations per XCD)
    with a random field and a per-cell force field: after 10 steps the moment
    storage agrees with FP32 population storage to 1e-6 in velocity in every
    member (two data paths of the same arithmetic; the FP32 path is pinned to
    the oracle elsewhere)."""
    log("mom32 vs fp32 populations, 256x96x40 nb=32, field force, 10 steps")
    nx, ny, nz, nb = 256, 96, 40, 32
    shape = (nb, nz, ny, nx)
    g = W.generator(57)
    rho0 = (1.0 + g.uniform(-1e-3, 1e-3, size=shape)).astype(np.float32)
    u0 = g.uniform(-0.03, 0.03, size=(3,) + shape).astype(np.float32)
    force = g.uniform(-1e-4, 1e-4, size=(3,) + shape).astype(np.float32)
    out = {}
    for st in ("mom32", "fp32"):
        lat = Lat(nx=nx, ny=ny, nz=nz, nbatch=nb, tau=0.6, storage=st)
        lat.set_force("field", field=force)
        lat.init(rho0, u0, dtype=torch.float32)
        lat.step(10)
        out[st] = lat.moments(dtype=torch.float32)[1].double()
        del lat
    a, b = out["mom32"], out["fp32"]
    err = [float(torch.linalg.vector_norm(a[:, m] - b[:, m]) / torch.linalg.vector_norm(b[:, m])) for m in range(nb)]
    log(f"  relative difference per member: max {max(err):.3e}, min {min(err):.3e}")
    assert max(err) < 1e-6


# (nbatch, nz, ny, nx): partial tiles in x and y within one z chunk; several x
# tiles and z chunks with partial last ones; one-cell axes
# (nb, nz, ny, nx).  The z chunk of the force tiles is chosen from the device's
# resident workgroups: the small shapes run one plane per chunk, the last two
# need more tiles than one generation holds, so their chunks march several
# planes through the rolling LDS window (ragged x, y and last z chunk).
PSI_SHAPES = [(2, 9, 10, 11), (1, 37, 9, 130), (1, 1, 1, 1), (1, 17, 1, 3), (2, 160, 99, 130), (1, 128, 128, 128)]


@pytest.mark.parametrize("shape", PSI_SHAPES)
@pytest.mark.parametrize("storage,tol", [("fp64", 1e-14), ("fp32", 1e-6)])
def test_pseudopotential_force_matches_oracle(torch, storage, tol, shape):
    log(f"pseudo-potential force {storage}, random density {shape}")
    nb, nz, ny, nx = shape
    rho = W.generator(61).uniform(0.1, 2.0, size=shape)
    ref = O.pseudopotential_force(rho, -6.0)
    lat = Lat(nx=nx, ny=ny, nz=nz, nbatch=nb, tau=1.0, storage=storage)
    F = lat.pseudopotential_force(-6.0, rho).double().cpu().numpy()
    err = np.abs(F - ref).max() / max(np.abs(ref).max(), 1.0)  # force scale |G| psi^2 ~ 1 (zero on one cell)
    log(f"  error {err:.3e}")
    assert err < tol


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16"])
def test_density_export_equals_moments(torch, storage):
    """The density-only export (velocity pointer NULL) equals the density of
    the full moment export bit for bit, with a per-cell force field (which
    enters only the velocity), walls, solid nodes and a ragged batch of two;
    and, in FP64, the oracle's density (eq. macroscopic)."""
    shape = (2, 5, 6, 37)
    g = W.generator(79)
    solid = (g.uniform(size=shape) < 0.08).astype(np.uint8)
    force = g.uniform(-1e-3, 1e-3, size=(3,) + shape)
    f0 = W.random_populations(shape, seed=80)
    f0[:, solid.astype(bool)] = 0.0
    lat = Lat(nx=37, ny=6, nz=5, nbatch=2, tau=0.7, storage=storage, wall=(0, 1, 1), solid=True)
    lat.set_solid(solid)
    lat.set_force("field", field=force)
    lat.load_populations(f0)
    lat.step(3)
    dt = torch.float64 if storage == "fp64" else torch.float32
    rho = lat.density(dtype=dt)
    assert torch.equal(rho, lat.moments(dtype=dt)[0])
    if storage == "fp64":
        ref = O.Lattice(37, 6, 5, nb=2, tau=0.7, wall=(0, 1, 1), solid=solid, force=force, extended=True)
        ref.load_populations(f0)
        ref.step(3)
        m = ~solid.astype(bool)
        assert rel(rho.cpu().numpy()[m], ref.moments()[0][m]) < 1e-14
    lat.close()


def test_fp64_static_droplet_steps(torch):
    """A small static droplet (24^3, radius 6, G = -6, tau = 1): 30 steps with
    the force refreshed from the density before every step, against the 80-bit
    oracle doing the same."""
    from paper_1905_10182_amd import studies
    log("fp64 static droplet 24^3, 30 steps")
    wl = W.static_droplet(24, 6.0)
    ref = O.Lattice(24, 24, 24, tau=wl["tau"], extended=True)
    ref.init(wl["rho"], wl["u"])
    for _ in range(30):
        ref.set_force(O.pseudopotential_force(ref.moments()[0], wl["g"], extended=True))
        ref.step(1)
    ref.set_force(O.pseudopotential_force(ref.moments()[0], wl["g"], extended=True))
    lat = Lat(nx=24, ny=24, nz=24, tau=wl["tau"], storage="fp64")
    rows, blew = studies.droplet_run(lat, wl, 30, out=open("/dev/null", "w"), every=lambda t: 30)
    assert blew is None
    rho, u = lat.moments()
    rr, ur = ref.moments()
    e_u = rel(u.cpu().numpy(), ur)
    e_r = rel(rho.cpu().numpy(), rr)
    log(f"  velocity {e_u:.3e} density {e_r:.3e}")
    assert e_u < 1e-12 and e_r < 1e-14


def test_fp64_four_rolls_mill_nz1_field_force(torch):
    """Four-rolls mill 16 x 16 x 1 (one node in z, periodic), per-node force
    field, 2000 steps from the analytic field."""
    log("fp64 four-rolls mill 16x16x1, 2000 steps")
    wl = W.four_rolls_mill(16)
    ref = O.Lattice(16, 16, 1, tau=wl["tau"], force=wl["force"], extended=True)
    ref.init(np.ones(wl["shape"]), wl["u_exact"])
    ref.step(2000)
    lat = Lat(nx=16, ny=16, nz=1, tau=wl["tau"], storage="fp64")
    lat.set_force("field", field=wl["force"])
    lat.init(np.ones(wl["shape"]), wl["u_exact"])
    lat.step(2000)
    _, u = lat.moments()
    _, ur = ref.moments()
    err = rel(u.cpu().numpy(), ur)
    log(f"  velocity {err:.3e}")
    assert err < 1e-12


def test_four_rolls_mill_convergence_fp64(torch):
    """Four-rolls mill at Re = 100, u0 = 1e-3 on the GPU (FP64): relative L2
    error of the steady velocity against the analytic field for N = 8..64,
    each grid run for two relaxation times from the analytic field.  The
    observed order between successive grids must be 2 within 0.1 (the paper
    prints 1.998)."""
    errs = []
    for n in (8, 16, 32, 64):
        wl = W.four_rolls_mill(n)
        lat = Lat(nx=n, ny=n, nz=1, tau=wl["tau"], storage="fp64")
        lat.set_force("field", field=wl["force"])
        lat.init(np.ones(wl["shape"]), wl["u_exact"])
        lat.step(int(2 * wl["t_relax"]))
        u = lat.moments()[1].cpu().numpy()
        errs.append(rel(u[:2], wl["u_exact"][:2]))
        log(f"  N={n}: error {errs[-1]:.4e}")
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(3)]
    log(f"  observed orders {rates}")
    assert all(1.9 < r < 2.1 for r in rates)


def test_fp64_sphere_channels_batch_force(torch):
    log("fp64 sphere channels 3x(40x20x16), 60 steps")
    wl = W.sphere_channels(3, nx=40, ny=20, nz=16, seed=77, rmin=2.0, rmax=4.0)
    solid = wl["solid"]
    nb, nz, ny, nx = wl["shape"]
    field = np.zeros((3,) + wl["shape"])
    field[0] = wl["fx"][:, None, None, None]
    ref = O.Lattice(nx, ny, nz, nb=nb, tau=wl["tau"], wall=wl["wall"], solid=solid, force=field, extended=True)
    rho0 = np.ones(wl["shape"])
    ref.init(rho0, np.zeros((3,) + wl["shape"]))
    ref.step(60)
    lat = Lat(nx=nx, ny=ny, nz=nz, nbatch=nb, tau=wl["tau"], storage="fp64", wall=wl["wall"], solid=True)
    lat.set_solid(solid)
    lat.set_force("batch", np.stack([wl["fx"], 0 * wl["fx"], 0 * wl["fx"]], axis=1))
    lat.init(None, None)
    lat.step(60)
    _, u = lat.moments()
    _, ur = ref.moments()
    err = fluid_rel(u.cpu().numpy(), ur, solid)
    log(f"  velocity {err:.3e}")
    assert err < 1e-12
    assert np.abs(u.cpu().numpy()[:, solid.astype(bool)]).max() == 0.0


# ---------------------------------------------------------------------------
# FP32 / 16-bit storage

def test_fp32_taylor_green_32(torch):
    log("fp32 TGV 32^3, 200 steps")
    ref, lat = tgv_pair(32, "fp32", 200)
    _, u = lat.moments()
    _, ur = ref.moments()
    err = rel(u.cpu().numpy(), ur)
    log(f"  velocity {err:.3e}")
    assert err < 1e-5


def test_fp32_poiseuille_config(torch):
    log("fp32 Poiseuille 32x16x16, 1000 steps")
    wl = W.poiseuille()
    nb, nz, ny, nx = wl["shape"]
    ref = O.Lattice(nx, ny, nz, tau=wl["tau"], wall=wl["wall"], force=wl["force"].reshape(3, 1, 1, 1, 1))
    ref.init(wl["rho"], wl["u"])
    ref.step(wl["steps"])
    lat = Lat(nx=nx, ny=ny, nz=nz, tau=wl["tau"], storage="fp32", wall=wl["wall"])
    lat.set_force("uniform", wl["force"])
    lat.init(wl["rho"], wl["u"])
    lat.step(wl["steps"])
    _, u = lat.moments()
    _, ur = ref.moments()
    err = rel(u.cpu().numpy(), ur)
    log(f"  velocity {err:.3e}")
    assert err < 1e-5


@pytest.mark.parametrize("storage,stochastic,bound", [("fp16", False, 1e-3), ("fp16", True, 1e-3),
                                                      ("bf16", False, 1e-2), ("bf16", True, 1e-2)])
def test_16bit_taylor_green_32_error(torch, storage, stochastic, bound):
    """Velocity error of 16-bit storage after 200 steps of TGV 32^3 (Re 1600)
    against the FP64 oracle: FP16 within the 1e-3 target with either
    rounding; BF16 (8-bit significand) within 1e-2."""
    log(f"{storage}{' stochastic rounding' if stochastic else ''} TGV 32^3, 200 steps")
    ref, lat = tgv_pair(32, storage, 200, stochastic=stochastic)
    _, u = lat.moments()
    _, ur = ref.moments()
    err = rel(u.cpu().numpy(), ur)
    log(f"  velocity error vs FP64 oracle {err:.3e}")
    assert err < bound


# ---------------------------------------------------------------------------
# full-size configurations, sampled

def sampled_one_step(torch, n, storage, nsample, seed, dims=None, re=1600.0, stochastic=False, force_amp=0.0):
    """One fused step; at nsample random cells s (every cell if nsample is
    None) the oracle collides the exported pre-collision populations P0[:, s]
    and each result f*_i must appear at P1[i, s + c_i].  force_amp > 0 adds a
    seeded per-cell force field, uniform in [-force_amp, force_amp] (FP32
    values, given to the oracle as they are)."""
    nx, ny, nz = dims or (n, n, n)
    wl = W.taylor_green(n, seed=1, re=re)
    rho, u = wl["rho"], wl["u"]
    if dims is not None:  # a periodic box cut from a larger vortex: still a valid state
        rho, u = rho[:, :nz, :ny, :nx], u[:, :, :nz, :ny, :nx]
    lat = Lat(nx=nx, ny=ny, nz=nz, tau=wl["tau"], storage=storage, stochastic=stochastic)
    field = None
    if force_amp > 0:
        dt = np.float64 if storage == "fp64" else np.float32
        field = W.generator(seed + 1000).uniform(-force_amp, force_amp, size=(3, 1, nz, ny, nx)).astype(dt)
        lat.set_force("field", field=field)
    lat.init(rho, u)
    del wl, rho, u
    if nsample is None:
        zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        s = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1)
    else:
        g = W.generator(seed)
        s = np.stack([g.integers(0, nx, nsample), g.integers(0, ny, nsample), g.integers(0, nz, nsample)], 1)
    P0 = lat.populations()
    lin0 = torch.as_tensor((s[:, 2] * ny + s[:, 1]) * nx + s[:, 0], device=P0.device)
    f0 = P0.reshape(27, -1)[:, lin0].cpu().numpy()
    del P0
    lat.step(1)
    P1 = lat.populations().reshape(27, -1)
    got = np.empty((27, len(s)))
    dims3 = np.array([nx, ny, nz])
    for i in range(27):
        d = (s + np.array([CX[i], CY[i], CZ[i]])) % dims3
        lin = torch.as_tensor((d[:, 2] * ny + d[:, 1]) * nx + d[:, 0], device=P1.device)
        got[i] = P1[i, lin].cpu().numpy()
    del P1
    F = None if field is None else field[:, 0, s[:, 2], s[:, 1], s[:, 0]].astype(np.float64)
    ref = O.collide_cells(f0, F, 1.0 / lat.params.tau)
    lat.close()
    return got, ref


def ulp16(h, storage):
    """Spacing of the stored 16-bit value at |h|: FP16 holds 256 h, BF16 holds h
    with an 8-bit significand."""
    if storage == "fp16":
        return np.spacing((np.abs(h) * 256).astype(np.float16)).astype(np.float64) / 256
    a = np.maximum(np.abs(h).astype(np.float32), np.float32(2.0 ** -126))
    return np.ldexp(1.0, np.floor(np.log2(a)).astype(np.int64) - 7)


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
@pytest.mark.parametrize("nx", [40, 42, 37, 264, 128])
def test_16bit_one_step_every_cell_is_rounded_oracle(torch, storage, nx):
    """Every post-collision population of one step equals the oracle's value
    rounded to nearest in the 16-bit format: |error| <= half a unit in the
    last place plus the FP32 arithmetic error (bounded by 2e-7 w_i; the FP32
    path itself stays below 1e-7 w_i).  nx = 40, 42 and 264 run the
    2-cells-per-lane kernel (one partial wave per row / a row over several
    waves), 128 it with a row of exactly one wave (the lane rotation is the
    periodic wrap), 37 the one-cell one."""
    log(f"{storage} one step, every cell, {nx}x12x10")
    got, ref = sampled_one_step(torch, max(nx, 64), storage, None, 0, dims=(nx, 12, 10), re=200.0)
    h_ref = ref - WGT[:, None]
    err = np.abs((got - WGT[:, None]) - h_ref)
    ulp = ulp16(h_ref, storage)
    log(f"  max error in ulps {(err / ulp).max():.3f}")
    assert np.all(err <= 0.5 * ulp + 2e-7 * WGT[:, None])


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
@pytest.mark.parametrize("nx", [40, 128, 37])
def test_16bit_one_step_strong_force_field_is_rounded_oracle(torch, storage, nx):
    """As the force-free case, with a per-cell force field of up to 2e-3 per
    component.  FP16 computes on its stored scale (256 h, with the force
    scaled alike), so a force term off by that scale, or dropped, moves
    populations by many units in the last place here."""
    log(f"{storage} one step, every cell, {nx}x12x10, force field |F| <= 2e-3")
    got, ref = sampled_one_step(torch, max(nx, 64), storage, None, 7, dims=(nx, 12, 10), re=200.0, force_amp=2e-3)
    h_ref = ref - WGT[:, None]
    err = np.abs((got - WGT[:, None]) - h_ref)
    ulp = ulp16(h_ref, storage)
    log(f"  max error in ulps {(err / ulp).max():.3f}")
    assert np.all(err <= 0.5 * ulp + 2e-7 * WGT[:, None])


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
@pytest.mark.parametrize("nx", [40, 37])
def test_16bit_stochastic_rounding_is_unbiased(torch, storage, nx):
    """Stochastic rounding: every stored population is one of the two 16-bit
    neighbours of the oracle's value (|error| <= 1 ulp + FP32 error), and the
    signed error averages to zero (unbiased) over the ~130k populations."""
    log(f"{storage} stochastic rounding, one step, {nx}x12x10")
    got, ref = sampled_one_step(torch, 64, storage, None, 0, dims=(nx, 12, 10), re=200.0, stochastic=True)
    h_ref = ref - WGT[:, None]
    d = (got - WGT[:, None]) - h_ref
    ulp = ulp16(h_ref, storage)
    assert np.all(np.abs(d) <= ulp + 2e-7 * WGT[:, None])
    big = np.abs(h_ref) > 1e-4 * WGT[:, None]  # skip values that are exact zeros
    mean = float(np.mean(d[big] / ulp[big]))
    frac_away = float(np.mean(np.abs(got - WGT[:, None])[big] > np.abs(h_ref)[big]))
    log(f"  mean signed error {mean:+.4f} ulp, rounded away from zero {frac_away:.3f}")
    assert abs(mean) < 0.01
    # calibration: a value at fractional position p between its two 16-bit
    # neighbours rounds away from zero with probability p, in every bin of p
    # and for every population index (each index has its own random operand)
    a = np.abs(h_ref)
    e = np.floor(np.log2(np.maximum(a * 256, 2.0 ** -14) if storage == "fp16" else np.maximum(a, 2.0 ** -126)))
    sp = np.ldexp(1.0, (e - 10).astype(np.int64)) / 256 if storage == "fp16" else np.ldexp(1.0, (e - 7).astype(np.int64))
    pos = (a - np.floor(a / sp) * sp) / sp
    away = np.abs(got - WGT[:, None]) > a
    use = big & (pos > 1e-3) & (pos < 1 - 1e-3)
    for lo in np.arange(0.0, 1.0, 0.2):
        sel = use & (pos >= lo) & (pos < lo + 0.2)
        fa, fp = float(np.mean(away[sel])), float(np.mean(pos[sel]))
        log(f"  position in [{lo:.1f}, {lo + 0.2:.1f}): {sel.sum()} values, rounded away {fa:.4f}, mean position {fp:.4f}")
        assert abs(fa - fp) < 0.02
    for i in range(27):
        sel = use[i]
        if sel.sum() >= 1000:
            assert abs(float(np.mean(away[i][sel] - pos[i][sel]))) < 0.04, i
    got2, _ = sampled_one_step(torch, 64, storage, None, 0, dims=(nx, 12, 10), re=200.0, stochastic=True)
    assert np.array_equal(got, got2)  # counter-based bits: reproducible


def test_full_size_taylor_green_256_fp32_sampled(torch):
    log("fp32 TGV 256^3 one step, 4096 sampled cells")
    got, ref = sampled_one_step(torch, 256, "fp32", 4096, seed=31)
    err = np.abs(got - ref) / WGT[:, None]
    log(f"  max |f* - oracle| / w = {err.max():.3e}")
    assert err.max() < 1e-6


def test_full_size_taylor_green_256_fp64_sampled(torch):
    """FP64 storage in the benchmark's configuration (TGV 256^3, 512-thread
    workgroups): every sampled post-collision population within 1e-12 of the
    oracle's collision of the exported state."""
    log("fp64 TGV 256^3 one step, 4096 sampled cells")
    got, ref = sampled_one_step(torch, 256, "fp64", 4096, seed=35)
    err = np.abs(got - ref) / WGT[:, None]
    log(f"  max |f* - oracle| / w = {err.max():.3e}")
    assert err.max() < 1e-12


def test_full_size_taylor_green_512_fp16_sampled(torch):
    """16-bit storage at 512^3: every sampled post-collision population is the
    oracle's value rounded to nearest FP16 (half an ulp plus the FP32
    arithmetic error)."""
    log("fp16 TGV 512^3 one step, 4096 sampled cells")
    got, ref = sampled_one_step(torch, 512, "fp16", 4096, seed=32)
    h_ref = ref - WGT[:, None]
    h_got = got - WGT[:, None]
    err = np.abs(h_got - h_ref)
    ulp = ulp16(h_ref, "fp16")
    log(f"  max error in FP16 ulps {(err / ulp).max():.3f}")
    assert np.all(err <= 0.5 * ulp + 2e-7 * WGT[:, None])


def test_full_size_taylor_green_512_bf16_sampled(torch):
    """BF16 storage at 512^3, the benchmark's 16-bit launch: every sampled
    post-collision population is the oracle's value rounded to nearest BF16."""
    log("bf16 TGV 512^3 one step, 4096 sampled cells")
    got, ref = sampled_one_step(torch, 512, "bf16", 4096, seed=33)
    h_ref = ref - WGT[:, None]
    err = np.abs((got - WGT[:, None]) - h_ref)
    ulp = ulp16(h_ref, "bf16")
    log(f"  max error in BF16 ulps {(err / ulp).max():.3f}")
    assert np.all(err <= 0.5 * ulp + 2e-7 * WGT[:, None])


SB = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}


def raw_populations(torch, lat, buf, cells, pre=True):
    """Populations at cells (n, 3: x, y, z) read directly from one of the
    lattice's two device buffers: (nbatch * nz * ny) row blocks, each the 27
    population rows of one lattice row, nx cells padded to 256 bytes, each
    value stored as h = f - w rho0 (FP16: 256 h).  A step stores each cell's post-collision
    populations at the cell itself and the next step pulls them, so the
    pre-collision f_i(x) of the state (pre=True) sits at x - c_i, and the
    post-collision values of the step that wrote the buffer (pre=False) at x.
    Returns (27, n) FP64."""
    storage = {0: "fp64", 1: "fp32", 2: "fp16", 3: "bf16"}[lat.storage]
    sb = SB[storage]
    _, nz, ny, nx = lat.shape
    nxp = -(-nx * sb // 256) * 256 // sb
    view = buf.view({"fp64": torch.float64, "fp32": torch.float32, "fp16": torch.float16,
                     "bf16": torch.bfloat16}[storage])
    dims3 = np.array([nx, ny, nz])
    idx = np.empty((27, len(cells)), np.int64)
    for i in range(27):
        d = (cells - np.array([CX[i], CY[i], CZ[i]])) % dims3 if pre else cells
        idx[i] = ((d[:, 2] * ny + d[:, 1]) * 27 + i) * nxp + d[:, 0]
    h = view[torch.as_tensor(idx.ravel(), device=buf.device)].double().cpu().numpy().reshape(27, -1)
    if storage == "fp16":
        h = h / 256.0
    return h + WGT[:, None] * lat.params.rho0


def test_raw_population_layout_matches_export(torch):
    """The raw-buffer reading used at the largest sizes equals the library's
    population export, for every storage type, before and after a step (the
    state alternates between the two buffers), and the post-collision values a
    step leaves at each cell equal the oracle's collision of its pre-collision
    populations."""
    for storage in ("fp64", "fp32", "fp16", "bf16"):
        lat = Lat(nx=37, ny=6, nz=5, tau=0.6, storage=storage)
        g = W.generator(77)
        lat.init(1.0 + 1e-3 * g.uniform(-1, 1, lat.shape), 0.05 * g.uniform(-1, 1, (3,) + lat.shape))
        zz, yy, xx = np.meshgrid(np.arange(5), np.arange(6), np.arange(37), indexing="ij")
        cells = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1)
        f0 = lat.populations().reshape(27, -1).cpu().numpy()
        assert np.array_equal(raw_populations(torch, lat, lat._a, cells), f0), storage
        lat.step(1)
        ref = lat.populations().reshape(27, -1).cpu().numpy()
        assert np.array_equal(raw_populations(torch, lat, lat._b, cells), ref), storage
        post = raw_populations(torch, lat, lat._b, cells, pre=False)
        err = np.abs(post - O.collide_cells(f0, None, 1.0 / lat.params.tau)) / WGT[:, None]
        assert err.max() < {"fp64": 1e-13, "fp32": 1e-6, "fp16": 1e-3, "bf16": 1e-2}[storage], storage
        lat.close()


# Population planes of 3 GiB: every in-plane byte offset past 2^31 (the top bit
# of the 32-bit offsets the kernels use), within the 4 GiB a plane may span.
LARGEST = [("fp16", (1024, 1024, 1536)), ("fp32", (1024, 1024, 768))]


@pytest.mark.parametrize("storage,dims", LARGEST)
def test_three_gib_planes_sampled(torch, storage, dims):
    """Initialisation, moments and one step on a lattice whose population
    planes are 3 GiB (162 GiB of populations), from a seeded per-cell random
    state (density 1 +- 1e-3, velocity components in +-0.05, drawn on the
    device): the moments of sampled cells against the oracle's from their
    stored populations, and their post-collision populations after the step
    against the oracle's collision (FP16: the rounded oracle value; FP32
    within 1e-6 w).  Samples include the last cells of the planes and their
    periodic neighbours at the planes' start."""
    nx, ny, nz = dims
    n = nx * ny * nz
    need = 2 * 27 * (n * SB[storage] + 4096) + 16 * n + (2 << 30)
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory, {free / 2**30:.0f} GiB free")
    log(f"{storage} {nx}x{ny}x{nz}: {27 * n * SB[storage] / 2**30:.0f} GiB of populations per buffer")
    lat = Lat(nx=nx, ny=ny, nz=nz, tau=0.6, storage=storage)
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(1536)
    rho = 1.0 + 2e-3 * (torch.rand(lat.shape, generator=gen, device="cuda:0") - 0.5)
    u = 0.1 * (torch.rand((3,) + lat.shape, generator=gen, device="cuda:0") - 0.5)
    lat.init(rho, u, dtype=torch.float32)
    del rho, u
    torch.cuda.empty_cache()
    g = W.generator(1536)
    corners = np.array([[x, y, z] for x in (0, nx - 1) for y in (0, ny - 1) for z in (0, nz - 1)])
    cells = np.concatenate([corners, np.stack([g.integers(0, nx, 2048), g.integers(0, ny, 2048),
                                               g.integers(0, nz, 2048)], 1)])
    f0 = raw_populations(torch, lat, lat._a, cells)
    rho_g, u_g = lat.moments(dtype=torch.float32)
    lin = torch.as_tensor((cells[:, 2] * ny + cells[:, 1]) * nx + cells[:, 0], device="cuda:0")
    rg = rho_g.reshape(-1)[lin].double().cpu().numpy()
    ug = u_g.reshape(3, -1)[:, lin].double().cpu().numpy()
    del rho_g, u_g
    torch.cuda.empty_cache()
    mom = [O.macroscopic(f0[:, k]) for k in range(len(cells))]
    assert np.abs(rg - np.array([m[0] for m in mom])).max() < 1e-6
    assert np.abs(ug - np.array([m[1] for m in mom]).T).max() < 1e-6
    lat.step(1)
    got = raw_populations(torch, lat, lat._b, cells, pre=False)
    ref = O.collide_cells(f0, None, 1.0 / lat.params.tau)
    lat.close()
    del lat
    torch.cuda.empty_cache()
    if storage == "fp16":
        h_ref = ref - WGT[:, None]
        err = np.abs((got - WGT[:, None]) - h_ref)
        ulp = ulp16(h_ref, "fp16")
        log(f"  max error in FP16 ulps {(err / ulp).max():.3f}")
        assert np.all(err <= 0.5 * ulp + 2e-7 * WGT[:, None])
    else:
        err = np.abs(got - ref) / WGT[:, None]
        log(f"  max |f* - oracle| / w = {err.max():.3e}")
        assert err.max() < 1e-6


def raw_moments(torch, lat, buf, cells):
    """The nine stored FP32 numbers (rho - rho0, u, (1 - omega) k4..k8) of
    moment storage at cells (n, 3), read from a device buffer: nine planes of
    (nbatch * nz * ny) rows of nx cells padded to 256 bytes, planes a further
    4 KiB apart, each cell's numbers at the cell itself.  Returns (9, n)."""
    _, nz, ny, nx = lat.shape
    nxp = -(-nx * 4 // 256) * 64
    pstride = nz * ny * nxp + 1024
    lin = (cells[:, 2] * ny + cells[:, 1]) * nxp + cells[:, 0]
    idx = np.arange(9)[:, None] * pstride + lin[None, :]
    return buf.view(torch.float32)[torch.as_tensor(idx.ravel(), device=buf.device)].double().cpu().numpy().reshape(9, -1)


def mom32_step_oracle(lat, cells, read):
    """The oracle's nine numbers after one step at cells, from the state's
    nine numbers read(points) at any points: each neighbour x - c_i's
    post-collision populations rebuilt from its numbers (eq.
    post_collision_central_moments_forcing, then the inverse transform),
    population i pulled, collided, and its density, velocity and relaxed
    k4..k8 formed."""
    _, nz, ny, nx = lat.shape
    dims3 = np.array([nx, ny, nz])
    om, rho0 = 1.0 / lat.params.tau, lat.params.rho0
    f = np.empty((27, len(cells)))
    for i in range(27):
        m = read((cells - np.array([CX[i], CY[i], CZ[i]])) % dims3)
        for j in range(len(cells)):
            k_post = O.post_collision(rho0 + m[0, j], m[4:9, j] / (1.0 - om), (0.0, 0.0, 0.0), om)
            f[i, j] = O.reconstruct_fast(m[1:4, j], k_post)[i]
    out = np.empty((9, len(cells)))
    for j in range(len(cells)):
        rho, u = O.macroscopic(f[:, j])
        out[:, j] = np.concatenate([[rho - rho0], u, (1.0 - om) * O.pre_collision(f[:, j], u)])
    return out


def test_mom32_raw_layout_matches_export_and_oracle(torch):
    """Moment storage read straight from its buffers: density and velocity
    equal the library's moment export, and one step's nine numbers at every
    cell match the oracle's step rebuilt from the previous buffer (1e-6)."""
    lat = Lat(nx=37, ny=6, nz=5, tau=0.6, storage="mom32")
    g = W.generator(78)
    lat.init(1.0 + 1e-3 * g.uniform(-1, 1, lat.shape), 0.05 * g.uniform(-1, 1, (3,) + lat.shape))
    zz, yy, xx = np.meshgrid(np.arange(5), np.arange(6), np.arange(37), indexing="ij")
    cells = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1)
    m0 = raw_moments(torch, lat, lat._a, cells)
    rho, u = lat.moments()
    assert np.array_equal(m0[0] + lat.params.rho0, rho.reshape(-1).cpu().numpy())
    assert np.array_equal(m0[1:4], u.reshape(3, -1).cpu().numpy())
    lat.step(1)
    got = raw_moments(torch, lat, lat._b, cells)
    ref = mom32_step_oracle(lat, cells, lambda pts: raw_moments(torch, lat, lat._a, pts))
    lat.close()
    log(f"  max |numbers - oracle| = {np.abs(got - ref).max():.3e}")
    assert np.abs(got - ref).max() < 1e-6


def test_mom32_three_gib_planes_sampled(torch):
    """Moment storage with 3 GiB planes (1024 x 1024 x 768, FP32 numbers, 54
    GiB per lattice): one step from a seeded per-cell random state drawn on
    the device, the nine numbers of 520 sampled cells (the planes' last cells
    and their periodic neighbours among them) against the oracle's step
    rebuilt from the stored numbers around each (1e-6)."""
    nx, ny, nz = 1024, 1024, 768
    n = nx * ny * nz
    need = 2 * 9 * (4 * n + 4096) + 16 * n + (2 << 30)
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory, {free / 2**30:.0f} GiB free")
    log(f"mom32 {nx}x{ny}x{nz}: {9 * n * 4 / 2**30:.0f} GiB of numbers per buffer")
    lat = Lat(nx=nx, ny=ny, nz=nz, tau=0.6, storage="mom32")
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(768)
    rho = 1.0 + 2e-3 * (torch.rand(lat.shape, generator=gen, device="cuda:0") - 0.5)
    u = 0.1 * (torch.rand((3,) + lat.shape, generator=gen, device="cuda:0") - 0.5)
    lat.init(rho, u, dtype=torch.float32)
    del rho, u
    torch.cuda.empty_cache()
    g = W.generator(768)
    corners = np.array([[x, y, z] for x in (0, nx - 1) for y in (0, ny - 1) for z in (0, nz - 1)])
    cells = np.concatenate([corners, np.stack([g.integers(0, nx, 512), g.integers(0, ny, 512),
                                               g.integers(0, nz, 512)], 1)])
    lat.step(1)
    got = raw_moments(torch, lat, lat._b, cells)
    ref = mom32_step_oracle(lat, cells, lambda pts: raw_moments(torch, lat, lat._a, pts))
    lat.close()
    del lat
    torch.cuda.empty_cache()
    log(f"  max |numbers - oracle| = {np.abs(got - ref).max():.3e}")
    assert np.abs(got - ref).max() < 1e-6


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_full_size_kolmogorov_384_sampled(torch, storage):
    """Kolmogorov flow at its full size, 384^3 (not a power of two: six waves per
    row in FP32, three in FP16), with the y-profile force: after three steps
    from the seeded state, one more step on 4096 sampled cells against the
    oracle's collision with each cell's force."""
    log(f"{storage} Kolmogorov 384^3, 3 + 1 steps, 4096 sampled cells")
    n = 384
    wl = W.kolmogorov(n)
    prof = wl["force_profile_y"]
    lat = Lat(nx=n, ny=n, nz=n, tau=wl["tau"], storage=storage)
    lat.set_force("profile_y", prof)
    lat.init(wl["rho"], wl["u"])
    del wl
    lat.step(3)
    g = W.generator(34)
    s = np.stack([g.integers(0, n, 4096), g.integers(0, n, 4096), g.integers(0, n, 4096)], 1)
    P0 = lat.populations().reshape(27, -1)
    f0 = P0[:, torch.as_tensor((s[:, 2] * n + s[:, 1]) * n + s[:, 0], device=P0.device)].cpu().numpy()
    del P0
    lat.step(1)
    P1 = lat.populations().reshape(27, -1)
    got = np.empty((27, len(s)))
    for i in range(27):
        d = (s + np.array([CX[i], CY[i], CZ[i]])) % n
        got[i] = P1[i, torch.as_tensor((d[:, 2] * n + d[:, 1]) * n + d[:, 0], device=P1.device)].cpu().numpy()
    del P1
    ref = O.collide_cells(f0, prof[s[:, 1]].T, 1.0 / lat.params.tau)
    lat.close()
    if storage == "fp32":
        err = np.abs(got - ref) / WGT[:, None]
        log(f"  max |f* - oracle| / w = {err.max():.3e}")
        assert err.max() < 1e-6
    else:
        h_ref = ref - WGT[:, None]
        err = np.abs((got - WGT[:, None]) - h_ref)
        ulp = ulp16(h_ref, storage)
        log(f"  max error in FP16 ulps {(err / ulp).max():.3f}")
        assert np.all(err <= 0.5 * ulp + 2e-7 * WGT[:, None])


# ---------------------------------------------------------------------------
# reductions, residual, checkpoint, failure detection

# axes of one or two cells: a cell is its own periodic neighbour along a
# one-cell axis, and 1 x 1 x 1 pulls every population from itself
DEGENERATE = [(1, 1, 1), (1, 5, 3), (7, 1, 1), (2, 1, 3), (1, 1, 4), (65, 1, 2)]


@pytest.mark.parametrize("dims", DEGENERATE)
@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16", "bf16"])
def test_degenerate_extents_match_oracle(torch, storage, dims):
    """One- and two-cell axes with a random non-equilibrium state and a
    per-cell force field: FP64 within 1e-13 of the 80-bit oracle after 4
    steps, FP32 within 1e-6 w_i, and the 16-bit formats one step from their
    stored state within half a unit in the last place (+ 2e-7 w_i) of the
    oracle's value.  A zero-step call changes nothing."""
    nx, ny, nz = dims
    shape = (1, nz, ny, nx)
    log(f"{storage} {nx}x{ny}x{nz}")
    g = W.generator(61)
    force = g.uniform(-1e-3, 1e-3, size=(3,) + shape)
    if storage != "fp64":
        force = force.astype(np.float32)
    lat = Lat(nx=nx, ny=ny, nz=nz, tau=0.7, storage=storage)
    lat.set_force("field", field=force)
    lat.load_populations(W.random_populations(shape, seed=62))
    f0 = lat.populations().cpu().numpy()  # the state as stored
    lat.step(0)
    assert np.array_equal(lat.populations().cpu().numpy(), f0) and lat.time == 0
    steps = 4 if storage in ("fp64", "fp32") else 1
    ref = O.Lattice(nx, ny, nz, tau=0.7, force=force.astype(np.float64), extended=storage == "fp64")
    ref.load_populations(f0)
    ref.step(steps)
    lat.step(steps)
    out = lat.populations().cpu().numpy().reshape(27, -1)
    fr = np.asarray(ref.f, np.float64).reshape(27, -1)
    lat.close()
    if storage == "fp64":
        assert np.abs(out - fr).max() / np.abs(fr).max() < 1e-13
    elif storage == "fp32":
        assert (np.abs(out - fr) / WGT[:, None]).max() < 1e-6
    else:
        h_ref = fr - WGT[:, None]
        err = np.abs((out - WGT[:, None]) - h_ref)
        assert np.all(err <= 0.5 * ulp16(h_ref, storage) + 2e-7 * WGT[:, None])


@pytest.mark.parametrize("dims,wall", [((5, 2, 3), (0, 1, 0)), ((2, 2, 2), (1, 1, 1)), ((1, 2, 2), (0, 1, 1)),
                                       ((3, 4, 1), (1, 1, 0))])
@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_narrowest_walled_channels_match_oracle(torch, storage, dims, wall):
    """Bounce-back walls across two-cell axes (the narrowest a walled axis may
    be), a solid node where the box allows one, a random state and a per-cell
    force field: 4 steps, FP64 within 1e-13 of the 80-bit oracle, FP32 within
    1e-6 w_i."""
    nx, ny, nz = dims
    shape = (1, nz, ny, nx)
    log(f"{storage} {nx}x{ny}x{nz} walls {wall}")
    g = W.generator(64)
    solid = np.zeros(shape, np.uint8)
    if nx * ny * nz >= 8:
        solid[0, 0, 0, 0] = 1
    f0 = W.random_populations(shape, seed=65)
    f0[:, solid.astype(bool)] = 0.0
    force = g.uniform(-1e-3, 1e-3, size=(3,) + shape)
    if storage != "fp64":
        force = force.astype(np.float32)
    lat = Lat(nx=nx, ny=ny, nz=nz, tau=0.7, storage=storage, wall=wall, solid=True)
    lat.set_solid(solid)
    lat.set_force("field", field=force)
    lat.load_populations(f0)
    f0 = lat.populations().cpu().numpy()  # the state as stored
    ref = O.Lattice(nx, ny, nz, tau=0.7, wall=wall, solid=solid, force=force.astype(np.float64),
                    extended=storage == "fp64")
    ref.load_populations(f0)
    ref.step(4)
    lat.step(4)
    out = lat.populations().cpu().numpy().reshape(27, -1)
    fr = np.asarray(ref.f, np.float64).reshape(27, -1)
    lat.close()
    if storage == "fp64":
        assert np.abs(out - fr).max() / np.abs(fr).max() < 1e-13
    else:
        assert (np.abs(out - fr) / WGT[:, None]).max() < 1e-6


@pytest.mark.parametrize("stochastic", [False, True])
@pytest.mark.parametrize("storage", ["fp16", "bf16"])
def test_16bit_walls_solids_force_one_step(torch, storage, stochastic):
    """16-bit storage on the masked kernel: walls in y and z, solid nodes, a
    per-cell force field, a ragged batch of two (70 cells per row: two cells
    per lane with a partial last wave), one step from the stored random state:
    every population within half a unit in the last place of the oracle's
    value (nearest rounding) or within one unit (stochastic), + 2e-7 w_i."""
    log(f"{storage} {'stochastic' if stochastic else 'nearest'} walls + solids 70x13x11 nb=2, one step")
    shape = (2, 11, 13, 70)
    g = W.generator(66)
    solid = (g.uniform(size=shape) < 0.08).astype(np.uint8)
    force = g.uniform(-1e-3, 1e-3, size=(3,) + shape).astype(np.float32)
    f0 = W.random_populations(shape, seed=67)
    f0[:, solid.astype(bool)] = 0.0
    lat = Lat(nx=70, ny=13, nz=11, nbatch=2, tau=0.7, storage=storage, wall=(0, 1, 1), solid=True,
              stochastic=stochastic)
    lat.set_solid(solid)
    lat.set_force("field", field=force)
    lat.load_populations(f0)
    f0 = lat.populations().cpu().numpy()  # the state as stored
    ref = O.Lattice(70, 13, 11, nb=2, tau=0.7, wall=(0, 1, 1), solid=solid, force=force.astype(np.float64))
    ref.load_populations(f0)
    ref.step(1)
    lat.step(1)
    fluid = ~solid.astype(bool).reshape(-1)
    out = lat.populations().cpu().numpy().reshape(27, -1)[:, fluid]
    fr = np.asarray(ref.f, np.float64).reshape(27, -1)[:, fluid]
    lat.close()
    h_ref = fr - WGT[:, None]
    err = np.abs((out - WGT[:, None]) - h_ref)
    ulp = ulp16(h_ref, storage)
    log(f"  max error in ulps {(err / ulp).max():.3f}")
    assert np.all(err <= (1.0 if stochastic else 0.5) * ulp + 2e-7 * WGT[:, None])


@pytest.mark.parametrize("dims", DEGENERATE)
def test_mom32_degenerate_extents_match_oracle(torch, dims):
    """Moment storage on one- and two-cell axes, from a random (rho, u) state
    with a per-cell force field: density and velocity within 1e-6 of the
    oracle after 4 steps."""
    nx, ny, nz = dims
    shape = (1, nz, ny, nx)
    log(f"mom32 {nx}x{ny}x{nz}")
    g = W.generator(63)
    rho = 1.0 + 1e-2 * g.uniform(-1, 1, shape)
    u = 0.05 * g.uniform(-1, 1, (3,) + shape)
    force = g.uniform(-1e-3, 1e-3, size=(3,) + shape).astype(np.float32)
    lat = Lat(nx=nx, ny=ny, nz=nz, tau=0.7, storage="mom32")
    lat.set_force("field", field=force)
    lat.init(rho, u)
    ref = O.Lattice(nx, ny, nz, tau=0.7, force=force.astype(np.float64))
    ref.init(rho, u)
    lat.step(4)
    ref.step(4)
    r, v = lat.moments()
    rr, vr = ref.moments()
    lat.close()
    assert np.abs(r.cpu().numpy() - rr).max() < 1e-6
    assert np.abs(v.cpu().numpy() - vr).max() < 1e-6


def test_reduce_matches_oracle_sums(torch):
    log("reduce vs oracle sums")
    shape = (2, 5, 6, 70)
    f0 = W.random_populations(shape, seed=41)
    lat = Lat(nx=70, ny=6, nz=5, nbatch=2, tau=0.9, storage="fp64")
    lat.load_populations(f0)
    r = lat.reduce()
    C = np.stack([CX, CY, CZ], 1).astype(float)
    for b in range(2):
        fb = f0[:, b].reshape(27, -1)
        assert abs(r[b, 0] / fb.sum() - 1) < 1e-14
        np.testing.assert_allclose(r[b, 1:4], fb.sum(axis=1) @ C, rtol=1e-12, atol=1e-13)
        assert r[b, 7] == fb.shape[1] and r[b, 6] == 0
    r2 = lat.reduce()
    assert np.array_equal(r, r2)  # fixed summation order


def test_periodic_momentum_gain_equals_force(torch):
    log("momentum bookkeeping fp64 periodic 64x8x8, 50 steps")
    F = np.array([2e-5, -1e-5, 3e-6])
    lat = Lat(nx=64, ny=8, nz=8, tau=0.7, storage="fp64")
    lat.set_force("uniform", F)
    lat.init(None, None)
    r0 = lat.reduce()
    lat.step(50)
    r1 = lat.reduce()
    ncell = 64 * 8 * 8
    np.testing.assert_allclose(r1[0, 1:4] - r0[0, 1:4], 50 * ncell * F, rtol=1e-11)
    assert abs(r1[0, 0] / r0[0, 0] - 1) < 1e-14


def test_residual_snapshot_semantics(torch):
    log("residual semantics")
    wl = W.taylor_green(24, re=200.0)
    lat = Lat(nx=24, ny=24, nz=24, tau=wl["tau"], storage="fp64", residual=True)
    lat.init(wl["rho"], wl["u"])
    _, ua = lat.moments()
    lat.reduce(snapshot=True)
    lat.step(3)
    _, ub = lat.moments()
    r = lat.reduce(residual=True, snapshot=True)
    a, b = ua.cpu().numpy(), ub.cpu().numpy()
    expect = np.linalg.norm(b - a) / np.linalg.norm(b)
    assert abs(r[0, 10] / expect - 1) < 1e-10


def test_checkpoint_restart_is_bitwise(torch):
    """save_state / restore_state: 40 steps in one go equal 20 steps, a
    checkpoint, a restore into a fresh handle and 20 more, bit for bit (every
    kernel is deterministic).  The FP64 population export/import path is
    exact up to one rounding of f - w rho0."""
    for storage in ("fp64", "fp32", "fp16"):
        log(f"checkpoint restart {storage} TGV 24^3")
        wl = W.taylor_green(24, re=400.0)
        A = Lat(nx=24, ny=24, nz=24, tau=wl["tau"], storage=storage)
        A.init(wl["rho"], wl["u"])
        A.step(40)
        B = Lat(nx=24, ny=24, nz=24, tau=wl["tau"], storage=storage)
        B.init(wl["rho"], wl["u"])
        B.step(20)
        blob, t = B.save_state()
        C = Lat(nx=24, ny=24, nz=24, tau=wl["tau"], storage=storage)
        C.restore_state(blob, t)
        C.step(20)
        assert C.time == 40
        assert torch.equal(A.populations(), C.populations())
    D = Lat(nx=24, ny=24, nz=24, tau=wl["tau"], storage="fp64")
    D.load_populations(B.populations())
    np.testing.assert_allclose(D.populations().cpu().numpy(), B.populations().cpu().numpy(), rtol=0, atol=1e-16)


def test_nonfinite_state_reports_unstable(torch):
    from paper_1905_10182_amd import cmlbm as B
    log("non-finite detection")
    f = WGT.reshape(27, 1, 1, 1, 1) * np.ones((27, 1, 4, 4, 64))
    f[3, 0, 1, 2, 5] = np.nan
    lat = Lat(nx=64, ny=4, nz=4, tau=0.7, storage="fp32")
    lat.load_populations(f)
    with pytest.raises(B.CmlbmError) as e:
        lat.reduce()
    assert e.value.code == B.EUNSTABLE
    r = lat.reduce(allow_unstable=True)
    assert r[0, 6] == 1 and r[0, 7] == 64 * 16


def test_device_copy_bitwise(torch):
    """The copy probe copies every byte, including a tail that is not a whole
    number of its 4 x 16-byte thread groups."""
    from paper_1905_10182_amd.cmlbm import device_copy
    g = torch.Generator(device="cuda:0").manual_seed(3)
    for n in (16 * 1024 * 4 + 12, 1000004 * 4):  # int32 counts: whole 16-byte units with ragged tails
        a = torch.randint(-2**31, 2**31 - 1, (n,), dtype=torch.int32, device="cuda:0", generator=g)
        b = torch.zeros_like(a)
        device_copy(b, a)
        torch.cuda.synchronize()
        assert torch.equal(a, b)


@pytest.mark.parametrize("planes", [27, 9])
def test_plane_copy_bitwise(torch, planes):
    """The plane copy copies every cell of every plane (a ragged last
    workgroup, planes spaced beyond their cells) and leaves the gaps between
    planes untouched."""
    from paper_1905_10182_amd.cmlbm import plane_copy
    g = torch.Generator(device="cuda:0").manual_seed(5)
    cells, stride = 1024 * 37 + 5, 1024 * 37 + 5 + 1031
    a = torch.randn((planes, stride), device="cuda:0", generator=g)
    b = torch.full_like(a, -7.0)
    plane_copy(b, a, planes, cells, stride)
    torch.cuda.synchronize()
    assert torch.equal(a[:, :cells], b[:, :cells])
    assert torch.all(b[:, cells:] == -7.0)


def test_row_block_copy_bitwise(torch):
    """The row-block copy copies every value of rows * 27 * row_len (a row
    length that is not a multiple of 64, a ragged last workgroup) and writes
    nothing beyond that span."""
    from paper_1905_10182_amd.cmlbm import row_block_copy
    g = torch.Generator(device="cuda:0").manual_seed(6)
    rows, row_len = 293, 101
    span = rows * 27 * row_len
    a = torch.randn(span + 777, device="cuda:0", generator=g)
    b = torch.full_like(a, -7.0)
    row_block_copy(b, a, rows, row_len)
    torch.cuda.synchronize()
    assert torch.equal(a[:span], b[:span])
    assert torch.all(b[span:] == -7.0)
