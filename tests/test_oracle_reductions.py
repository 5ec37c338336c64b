"""Pins of the oracle's global monitors (oracle.reductions: mass, momentum,
kinetic energy, max |u|, sum |u|^2, residual, fluid and non-finite counts)
against closed forms fixed by the inputs and by the method, not against the
oracle's own formulas.

- A lattice initialised at the equilibrium f^eq(rho1, U) of eq. eq:truncation
  has zeroth and first moments rho1 and rho1 U (they are conserved moments of
  the equilibrium), so every monitor has a closed form in (rho1, U, N).  rho1
  differs from 1, so a weight of rho0 instead of rho fails; the 1/2 of the
  kinetic energy, the square of |u| and the square root of max |u| all show.
- With a force F in effect, eq. macroscopic gives u = U + F / (2 rho1) but
  sum f c = rho1 U: the kinetic energy and max |u| take the half-force
  velocity, the momentum sum does not.
- On a periodic lattice the momentum sum gains exactly sum F per step (the
  post-collision first moments are F/2 above the pre-collision ones, eq.
  post_collision_central_moments_forcing) and the mass does not change.
- The kinetic energy of the small-amplitude z-invariant Taylor-Green vortex
  decays as exp(-4 nu k^2 t) (an exact Navier-Stokes solution).
"""
import math

import numpy as np

import oracle as O
import workloads as W

SHAPE = (2, 4, 5, 6)  # nb, nz, ny, nx
N = 4 * 5 * 6
RHO1 = np.array([1.07, 0.93])
U1 = np.array([[0.03, -0.02, 0.01], [-0.01, 0.04, 0.02]])


def uniform_lattice(rho1, U, solid=None, force=None):
    L = O.Lattice(SHAPE[3], SHAPE[2], SHAPE[1], nb=SHAPE[0], tau=0.7, solid=solid, force=force)
    rho = np.broadcast_to(np.asarray(rho1)[:, None, None, None], SHAPE)
    u = np.broadcast_to(np.asarray(U).T[:, :, None, None, None], (3,) + SHAPE)
    L.init(rho, u)
    return L


def close(a, b, rtol=1e-13):
    np.testing.assert_allclose(np.asarray(a, np.float64), np.asarray(b, np.float64), rtol=rtol, atol=0)


def test_uniform_state_closed_forms():
    red = uniform_lattice(RHO1, U1).reductions()
    for b in range(2):
        r, U = RHO1[b], U1[b]
        d = red[b]
        close(d["mass"], N * r)
        close(d["mom"], N * r * U)
        close(d["ke"], N * r * (U @ U) / 2)
        close(d["umax"], math.sqrt(U @ U))
        close(d["u2"], N * (U @ U))
        assert d["fluid"] == N and d["nonfinite"] == 0
        assert d["du2"] == 0 and d["residual"] == 0


def test_half_force_velocity_enters_energy_not_momentum():
    F = np.array([[2e-3, -1e-3, 5e-4], [-4e-3, 3e-3, 1e-3]])
    field = np.broadcast_to(F.T[:, :, None, None, None], (3,) + SHAPE)
    red = uniform_lattice(RHO1, U1, force=field).reductions()
    for b in range(2):
        r, U = RHO1[b], U1[b]
        uh = U + F[b] / (2 * r)
        d = red[b]
        close(d["mom"], N * r * U, rtol=1e-12)
        close(d["ke"], N * r * (uh @ uh) / 2)
        close(d["umax"], math.sqrt(uh @ uh))
        close(d["u2"], N * (uh @ uh))


def test_solid_cells_are_excluded():
    solid = np.zeros(SHAPE, np.uint8)
    solid[0, 1, 2, :4] = 1
    solid[1, :, 0, 0] = 1
    red = uniform_lattice(RHO1, U1, solid=solid).reductions()
    for b in range(2):
        nf = N - int(solid[b].sum())
        r, U = RHO1[b], U1[b]
        assert red[b]["fluid"] == nf
        close(red[b]["mass"], nf * r)
        close(red[b]["ke"], nf * r * (U @ U) / 2)


def test_residual_of_two_uniform_states():
    Ua = U1
    Ub = U1 + np.array([[1e-3, 2e-3, -1e-3], [0.0, -5e-3, 4e-3]])
    A = uniform_lattice(RHO1, Ua)
    snap = A.moments()[1]
    red = uniform_lattice(RHO1, Ub).reductions(u_snapshot=snap)
    for b in range(2):
        dv = Ub[b] - Ua[b]
        close(red[b]["du2"], N * (dv @ dv), rtol=1e-11)
        close(red[b]["residual"], math.sqrt(dv @ dv) / math.sqrt(Ub[b] @ Ub[b]), rtol=1e-11)


def test_nonfinite_cell_is_counted_in_its_member_only():
    L = uniform_lattice(RHO1, U1)
    L.f[5, 1, 2, 3, 4] = np.nan
    red = L.reductions()
    assert red[1]["nonfinite"] == 1 and red[0]["nonfinite"] == 0
    close(red[0]["ke"], N * RHO1[0] * (U1[0] @ U1[0]) / 2)


def test_momentum_gains_force_and_mass_is_conserved():
    F = np.array([3e-5, -2e-5, 1e-5])
    rng = np.random.Generator(np.random.PCG64(5))
    L = O.Lattice(6, 5, 4, nb=1, tau=0.65, force=np.broadcast_to(F[:, None, None, None, None], (3, 1, 4, 5, 6)))
    u = rng.uniform(-0.02, 0.02, size=(3, 1, 4, 5, 6))
    L.init(1.0 + rng.uniform(-0.01, 0.01, size=(1, 4, 5, 6)), u)
    r0 = L.reductions()[0]
    L.step(7)
    r1 = L.reductions()[0]
    np.testing.assert_allclose(r1["mom"] - r0["mom"], 7 * N * F, rtol=1e-10)
    assert abs(r1["mass"] / r0["mass"] - 1) < 1e-14


def test_kinetic_energy_decay_of_taylor_green_2d():
    """ke(t2) / ke(t1) = exp(-4 nu k^2 (t2 - t1)) to the second-order error of
    the lattice (about 2% of the rate at n = 32, tau = 0.6)."""
    n, tau, u0, t1, t2 = 32, 0.6, 1e-3, 100, 300
    k = 2 * math.pi / n
    c = np.arange(n) * k
    u = np.zeros((3, 1, 1, n, n))
    u[0, 0, 0] = u0 * np.cos(c)[:, None] * np.sin(c)[None, :]
    u[1, 0, 0] = -u0 * np.sin(c)[:, None] * np.cos(c)[None, :]
    rho = np.ones((1, 1, n, n))
    rho[0, 0] = 1 - 3 * u0 ** 2 / 4 * (np.cos(2 * c)[None, :] + np.cos(2 * c)[:, None])
    L = O.Lattice(n, n, 1, tau=tau)
    L.init(rho, u)
    L.step(t1)
    e1 = L.reductions()[0]["ke"]
    L.step(t2 - t1)
    e2 = L.reductions()[0]["ke"]
    nu = (tau - 0.5) / 3
    rate = -math.log(e2 / e1) / (t2 - t1) / (4 * nu * k * k)
    assert abs(rate - 1) < 0.03, rate
    # and the kinetic energy of the initial field is the closed form sum rho |u|^2 / 2
    L.init(rho, u)
    close(L.reductions()[0]["ke"], (rho[0] * (u[:2, 0] ** 2).sum(axis=0)).sum() / 2, rtol=1e-12)


def test_blow_up_is_detected():
    """A Taylor-Green vortex at u0 = 0.3 (Mach 0.52) and tau = 0.5005 on 32^3
    is unstable: the oracle's state turns non-finite, and the reductions'
    non-finite count fires then and not before (checked every 5 steps)."""
    wl = W.taylor_green(32, seed=1, u0=0.3)
    lat = O.Lattice(32, 32, 32, tau=0.5005)
    lat.init(wl["rho"], wl["u"])
    fired = None
    for k in range(5, 401, 5):
        lat.step(5)
        with np.errstate(invalid="ignore", over="ignore"):  # sums over the non-finite cells
            r = lat.reductions()[0]
        if r["nonfinite"]:
            fired = k
            break
        assert np.isfinite(r["ke"]) and r["fluid"] == 32 ** 3
    assert fired is not None and 100 < fired <= 400, fired
