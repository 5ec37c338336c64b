"""Pins of the FP64 CPU oracle against facts fixed by the paper and by
mathematics (not against the oracle itself).

Paper: De Rosis, Huang & Coreixas, PRE 2019, arXiv:1905.10182, Sec. II.
Printed tables live in tests/golden/central_moment_tables.json with their
equation labels.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "central_moment_tables.json")))
CS2 = 1.0 / 3.0
CX, CY, CZ, WGT, OPP = O.constants()
C = np.stack([CX, CY, CZ], axis=1).astype(float)


def table_vector(entries, rho=None, F=None, k=None, omega=None):
    out = np.zeros(27)
    for j, (kind, comp, coef, p) in entries.items():
        if kind == "rho":
            x = rho
        elif kind == "F":
            x = F[comp]
        else:
            x = (1.0 - omega) * k[comp]
        out[int(j)] = coef * x * CS2 ** p
    return out


def product_feq(rho, u):
    """Tensor-product form of the complete D3Q27 Hermite equilibrium:
    w_i rho prod_a [1 + c_a u_a / cs^2 + (c_a^2 - cs^2) u_a^2 / (2 cs^4)]."""
    out = np.empty(27)
    for i in range(27):
        p = 1.0
        for a in range(3):
            c = C[i, a]
            p *= 1 + c * u[a] / CS2 + (c * c - CS2) * u[a] ** 2 / (2 * CS2 ** 2)
        out[i] = WGT[i] * rho * p
    return out


@pytest.fixture(scope="module")
def cells():
    rho, u = W.random_cells(20, seed=7, umax=0.2)
    return list(zip(rho, u))


# ---------------------------------------------------------------------------
# lattice

def test_lattice_matches_printed_list():
    g = GOLD["lattice"]
    assert list(CX) == g["cx"] and list(CY) == g["cy"] and list(CZ) == g["cz"]
    expect = [8 / 27] + [2 / 27] * 6 + [1 / 54] * 12 + [1 / 216] * 8
    np.testing.assert_allclose(WGT, expect, rtol=0, atol=1e-17)
    for i in range(27):
        assert np.all(C[OPP[i]] == -C[i])


def test_weights_quadrature_moments():
    # isotropy of the D3Q27 quadrature with cs^2 = 1/3
    assert abs(WGT.sum() - 1) < 1e-15
    np.testing.assert_allclose(WGT @ C, 0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", WGT, C, C), CS2 * np.eye(3), atol=1e-16)
    assert abs(np.sum(WGT * C[:, 0] ** 2 * C[:, 1] ** 2) - CS2 ** 2) < 1e-16
    assert abs(np.sum(WGT * C[:, 0] ** 2 * C[:, 1] ** 2 * C[:, 2] ** 2) - CS2 ** 3) < 1e-16


# ---------------------------------------------------------------------------
# equilibrium (eq. eq:truncation) and its central moments

def test_feq_equals_tensor_product_form(cells):
    for rho, u in cells:
        np.testing.assert_allclose(O.feq(rho, u), product_feq(rho, u), rtol=1e-14, atol=1e-16)


def test_feq_conserved_moments(cells):
    for rho, u in cells:
        f = O.feq(rho, u)
        assert abs(f.sum() - rho) < 1e-14
        np.testing.assert_allclose(f @ C, rho * u, atol=1e-15)
        # complete equilibrium: second moments are exactly rho (u u + cs^2 I)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", f, C, C), rho * (np.outer(u, u) + CS2 * np.eye(3)),
                                   atol=1e-15)


def test_equilibrium_central_moments_are_printed_table(cells):
    """Galilean invariance of the complete equilibrium: T^T f^eq is the
    velocity-free table of eq. equil_central_moments6 for every u."""
    for rho, u in cells:
        k = O.central_moments(u, O.feq(rho, u))
        np.testing.assert_allclose(k, table_vector(GOLD["equilibrium"]["entries"], rho=rho), atol=1e-15)


def test_second_order_equilibrium_is_not_galilean_invariant():
    # control: truncating the equilibrium at H^(2) leaves velocity-dependent CMs
    rho, u = 1.0, np.array([0.1, -0.05, 0.07])
    f2 = np.array([WGT[i] * rho * (1 + C[i] @ u / CS2 + ((C[i] @ u) ** 2 - CS2 * u @ u) / (2 * CS2 ** 2))
                   for i in range(27)])
    k = O.central_moments(u, f2)
    assert np.abs(k - table_vector(GOLD["equilibrium"]["entries"], rho=rho)).max() > 1e-4


# ---------------------------------------------------------------------------
# forcing (eq. forcing) and its central moments

def test_forcing_is_velocity_gradient_of_equilibrium(cells):
    """Reading of eq. forcing with F a force density: F . grad_u f^eq(rho=1, u),
    checked by central differences of the independent product form."""
    g = W.generator(3)
    for rho, u in cells:
        F = g.uniform(-1, 1, 3)
        h = 1e-5
        num = np.zeros(27)
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            num += F[a] * (product_feq(1.0, u + e) - product_feq(1.0, u - e)) / (2 * h)
        np.testing.assert_allclose(O.forcing(u, F), num, atol=1e-10)


def test_forcing_central_moments_are_printed_table(cells):
    g = W.generator(4)
    for rho, u in cells:
        F = g.uniform(-1e-2, 1e-2, 3)
        R = O.central_moments(u, O.forcing(u, F))
        np.testing.assert_allclose(R, table_vector(GOLD["forcing_sixth_order"]["entries"], F=F), atol=1e-17)


def test_guo_truncation_is_not_galilean_invariant():
    # control: keeping only H^(1), H^(2) of the forcing leaves R10 velocity-dependent
    # (the first table of the forcing discussion in Sec. II)
    u = np.array([0.1, 0.05, -0.02])
    F = np.array([1e-3, 2e-3, -1e-3])
    guo = np.array([WGT[i] * (F @ C[i] / CS2 + ((F @ C[i]) * (u @ C[i]) - CS2 * F @ u) / CS2 ** 2)
                    for i in range(27)])
    R = O.central_moments(u, guo)
    expect10 = 2 * F[0] * CS2 - F[0] * u[1] ** 2 - 2 * F[1] * u[0] * u[1] - F[0] * u[2] ** 2 - 2 * F[2] * u[0] * u[2]
    assert abs(R[10] - expect10) < 1e-15
    assert abs(R[16] - (-F[2] * u[0] * u[1] - F[1] * u[0] * u[2] - F[0] * u[1] * u[2])) < 1e-15


# ---------------------------------------------------------------------------
# basis (eq. basis) and its inverse (eq. system)

def test_basis_determinant_is_velocity_free():
    """|det T-bar| = 2^27 (three 1D Vandermonde factors of det 2) times 96 (the
    basis combinations: 3 for (k7, k8, k9), 2^3 for the third-order pairs,
    4 for (k17, k18, k19)) = 3 * 2^32, for every u."""
    g = W.generator(5)
    for _ in range(10):
        u = g.uniform(-0.3, 0.3, 3)
        d = abs(np.linalg.det(O.basis(u)))
        assert abs(d / (3 * 2 ** 32) - 1) < 1e-12


def test_fast_reconstruction_equals_linear_solve():
    g = W.generator(6)
    for _ in range(20):
        u = g.uniform(-0.3, 0.3, 3)
        k = g.normal(size=27)
        a = O.reconstruct_literal(u, k)
        b = O.reconstruct_fast(u, k)
        np.testing.assert_allclose(b, a, atol=1e-13)
        np.testing.assert_allclose(O.central_moments(u, b), k, atol=1e-13)


# ---------------------------------------------------------------------------
# collision

def test_collide_literal_equals_closed_form():
    g = W.generator(8)
    for _ in range(30):
        f = W.random_populations((), seed=int(g.integers(1 << 30))).ravel()
        F = g.uniform(-1e-2, 1e-2, 3)
        omega = g.uniform(0.5, 1.95)
        np.testing.assert_allclose(O.collide_closed(f, F, omega), O.collide_literal(f, F, omega), atol=2e-15)


def test_post_collision_moments_are_printed_table():
    g = W.generator(9)
    for _ in range(10):
        f = W.random_populations((), seed=int(g.integers(1 << 30))).ravel()
        F = g.uniform(-1e-2, 1e-2, 3)
        omega = g.uniform(0.5, 1.95)
        rho, u = O.macroscopic(f, F)
        k = O.central_moments(u, f)
        ks = O.central_moments(u, O.collide_closed(f, F, omega))
        expect = table_vector(GOLD["post_collision_forced"]["entries"], rho=rho, F=F, k=k, omega=omega)
        np.testing.assert_allclose(ks, expect, atol=2e-15)


def test_pre_collision_first_moments_are_minus_half_force():
    # with u from eq. macroscopic, sum f (c - u) = -F/2
    f = W.random_populations((), seed=11).ravel()
    F = np.array([3e-3, -1e-3, 2e-3])
    rho, u = O.macroscopic(f, F)
    np.testing.assert_allclose(O.central_moments(u, f)[1:4], -F / 2, atol=1e-16)


def test_equilibrium_is_fixed_point_without_force(cells):
    for rho, u in cells:
        fe = O.feq(rho, u)
        for omega in (0.6, 1.0, 1.7):
            np.testing.assert_allclose(O.collide_closed(fe, np.zeros(3), omega), fe, atol=1e-15)


def test_mass_and_momentum_with_half_force():
    """Sum f* = sum f and sum f* c = sum f c + F (k1..3* = F/2 with the
    half-force velocity)."""
    g = W.generator(12)
    for _ in range(20):
        f = W.random_populations((), seed=int(g.integers(1 << 30))).ravel()
        F = g.uniform(-1e-2, 1e-2, 3)
        fs = O.collide_closed(f, F, g.uniform(0.5, 1.95))
        assert abs(fs.sum() - f.sum()) < 1e-15
        np.testing.assert_allclose(fs @ C, f @ C + F, atol=1e-16)


def test_omega_one_reduces_to_equilibrium_plus_half_forcing():
    # omega = 1: every moment is equilibrated, so f* = f^eq + F_i / 2, the BGK
    # form of eq. collision at omega = 1
    g = W.generator(13)
    for _ in range(10):
        f = W.random_populations((), seed=int(g.integers(1 << 30))).ravel()
        F = g.uniform(-1e-2, 1e-2, 3)
        rho, u = O.macroscopic(f, F)
        np.testing.assert_allclose(O.collide_closed(f, F, 1.0), product_feq(rho, u) + 0.5 * O.forcing(u, F),
                                   atol=1e-15)


def test_shear_moments_relax_with_omega():
    # a pure shear perturbation at rest, d_i = w_i cx cy (1 - cz^2): its only
    # non-zero central moment is k4, which must come out as (1 - omega) k4
    f = product_feq(1.0, np.zeros(3))
    d = np.array([WGT[i] * C[i, 0] * C[i, 1] * (1 - C[i, 2] ** 2) for i in range(27)]) * 1e-3
    k = O.central_moments(np.zeros(3), d)
    assert abs(k[4]) > 1e-5 and np.abs(np.delete(k, 4)).max() < 1e-18
    omega = 1.3
    fs = O.collide_closed(f + d, np.zeros(3), omega)
    np.testing.assert_allclose(fs - f, (1 - omega) * d, atol=1e-16)


# ---------------------------------------------------------------------------
# lattice level

def test_literal_and_closed_lattices_agree():
    g = W.generator(14)
    shape = (1, 3, 4, 5)
    f0 = W.random_populations(shape, seed=15)
    force = g.uniform(-1e-3, 1e-3, (3,) + shape)
    A = O.Lattice(5, 4, 3, tau=0.7, wall=(0, 1, 0), force=force)
    B = O.Lattice(5, 4, 3, tau=0.7, wall=(0, 1, 0), force=force)
    A.load_populations(f0)
    B.load_populations(f0)
    A.step(5, "literal")
    B.step(5, "closed")
    np.testing.assert_allclose(A.f, B.f, atol=1e-14)


def test_periodic_mass_momentum_bookkeeping():
    shape = (1, 6, 5, 4)
    g = W.generator(16)
    f0 = W.random_populations(shape, seed=17)
    force = g.uniform(-1e-3, 1e-3, (3,) + shape)
    L = O.Lattice(4, 5, 6, tau=0.9, force=force)
    L.load_populations(f0)
    m0 = L.f.sum()
    p0 = (L.f.reshape(27, -1).sum(axis=1) @ C)
    L.step(10)
    assert abs(L.f.sum() / m0 - 1) < 1e-14
    np.testing.assert_allclose((L.f.reshape(27, -1).sum(axis=1) @ C), p0 + 10 * force.sum(axis=(1, 2, 3, 4)),
                               atol=1e-13)


def test_bounce_back_conserves_mass():
    shape = (1, 4, 6, 5)
    f0 = W.random_populations(shape, seed=18)
    solid = np.zeros(shape, np.uint8)
    solid[0, 1, 2, 2] = 1
    f0[:, solid.astype(bool)] = 0
    L = O.Lattice(5, 6, 4, tau=0.8, wall=(0, 1, 1), solid=solid)
    L.load_populations(f0)
    m0 = L.f.sum()
    L.step(20)
    assert abs(L.f.sum() / m0 - 1) < 1e-14


def poiseuille_series(y, t, F, nu, H, nterms=200):
    """Start-up of body-force channel flow between walls at y' = 0 and H,
    fluid at rest at t = 0 (Fourier series of the diffusion equation)."""
    u = F / (2 * nu) * y * (H - y)
    for n in range(1, 2 * nterms, 2):
        u -= 4 * F * H * H / (nu * math.pi ** 3 * n ** 3) * np.sin(n * math.pi * y / H) * math.exp(
            -n * n * math.pi ** 2 * nu * t / (H * H))
    return u


def test_poiseuille_startup_matches_series():
    """Body-force channel (walls halfway between nodes, H = ny) against the
    analytic start-up series of the Navier-Stokes equations; the channel is
    invariant in x and z, so one column carries the solution."""
    wl = W.poiseuille()
    ny, tau, fx = wl["shape"][2], wl["tau"], wl["force"][0]
    nu = (tau - 0.5) / 3
    L = O.Lattice(1, ny, 1, tau=tau, wall=(0, 1, 0), force=np.array([fx, 0, 0]).reshape(3, 1, 1, 1, 1))
    L.init(1.0, np.zeros((3, 1, 1, ny, 1)))
    L.step(wl["steps"])
    _, u = L.moments()
    ux = u[0, 0, 0, :, 0]
    y = np.arange(ny) + 0.5
    ref = poiseuille_series(y, wl["steps"], fx, nu, ny)
    err = np.linalg.norm(ux - ref) / np.linalg.norm(ref)
    assert err < 3e-3, err
    assert np.abs(u[1:]).max() < 1e-12  # no cross-flow beyond round-off


def test_poiseuille_steady_state_is_parabolic():
    """At steady state the bulk profile satisfies nu u'' = -F exactly (second
    difference of a parabola), and the profile is symmetric."""
    ny, tau, fx = 16, 0.8, 1e-6
    nu = (tau - 0.5) / 3
    L = O.Lattice(1, ny, 1, tau=tau, wall=(0, 1, 0), force=np.array([fx, 0, 0]).reshape(3, 1, 1, 1, 1))
    L.init(1.0, np.zeros((3, 1, 1, ny, 1)))
    L.step(20000)
    _, u = L.moments()
    ux = u[0, 0, 0, :, 0]
    d2 = ux[2:] - 2 * ux[1:-1] + ux[:-2]
    np.testing.assert_allclose(d2, -fx / nu, rtol=1e-6)
    np.testing.assert_allclose(ux, ux[::-1], rtol=1e-12)
    umax = fx * ny * ny / (8 * nu)
    assert abs(ux.max() / umax - 1) < 0.02


def shear_wave_rate(n, tau, amp=1e-4, t1=100, t2=400):
    """Decay rate of u_x(y) = A sin(2 pi y / n), measured between t1 and t2
    (after the start-up layer), in units of nu k^2."""
    y = np.arange(n)
    s = np.sin(2 * math.pi * y / n)
    u = np.zeros((3, 1, 1, n, 1))
    u[0, 0, 0, :, 0] = amp * s
    L = O.Lattice(1, n, 1, tau=tau)
    L.init(1.0, u)
    L.step(t1)
    a = L.moments()[1][0, 0, 0, :, 0] @ s
    L.step(t2 - t1)
    b = L.moments()[1][0, 0, 0, :, 0] @ s
    nu = (tau - 0.5) / 3
    return -math.log(b / a) / (t2 - t1) / (nu * (2 * math.pi / n) ** 2)


def test_shear_wave_viscosity():
    """omega = (nu / cs^2 + 1/2)^-1: the measured decay rate of a shear wave
    tends to nu k^2 at second order in the resolution."""
    for tau in (0.6, 0.8):
        e = [abs(shear_wave_rate(n, tau) - 1) for n in (16, 32, 64)]
        assert e[2] < 1e-3
        assert 3.5 < e[0] / e[1] < 4.5 and 3.5 < e[1] / e[2] < 4.5, e


def tgv2d_rate(n, tau=0.6, u0=1e-3, t1=100, t2=400):
    """Energy decay rate of the z-invariant Taylor-Green vortex
    u = u0 (sin kx cos ky, -cos kx sin ky, 0) with its pressure field
    rho = 1 - 3 u0^2/4 (cos 2kx + cos 2ky), between t1 and t2, in units of
    4 nu k^2."""
    k = 2 * math.pi / n
    c = np.arange(n) * k
    u = np.zeros((3, 1, 1, n, n))
    u[0, 0, 0] = u0 * np.cos(c)[:, None] * np.sin(c)[None, :]  # axes (y, x)
    u[1, 0, 0] = -u0 * np.sin(c)[:, None] * np.cos(c)[None, :]
    rho = np.ones((1, 1, n, n))
    rho[0, 0] = 1 - 3 * u0 ** 2 / 4 * (np.cos(2 * c)[None, :] + np.cos(2 * c)[:, None])
    L = O.Lattice(n, n, 1, tau=tau)
    L.init(rho, u)
    L.step(t1)
    e0 = (L.moments()[1][:2] ** 2).sum()
    L.step(t2 - t1)
    e1 = (L.moments()[1][:2] ** 2).sum()
    nu = (tau - 0.5) / 3
    return -math.log(e1 / e0) / (t2 - t1) / (4 * nu * k * k)


def test_taylor_green_2d_energy_decay():
    """The z-invariant Taylor-Green vortex is an exact Navier-Stokes solution
    with E(t) = E0 exp(-4 nu k^2 t); the measured rate converges to it at
    second order."""
    for tau in (0.6, 0.8):
        e = [abs(tgv2d_rate(n, tau) - 1) for n in (16, 32, 64)]
        assert e[2] < 2e-4
        assert 3.5 < e[0] / e[1] < 4.5 and 3.5 < e[1] / e[2] < 4.5, e


def test_galilean_invariance_of_decay():
    # a uniform background velocity leaves the shear-wave decay rate unchanged to O(k^2)
    n, tau, amp, U = 32, 0.6, 1e-4, 0.05
    y = np.arange(n)
    rates = []
    for bg in (0.0, U):
        u = np.zeros((3, 1, 1, n, 1))
        u[0, 0, 0, :, 0] = amp * np.sin(2 * math.pi * y / n)
        u[2] = bg
        L = O.Lattice(1, n, 1, tau=tau)
        L.init(1.0, u)
        L.step(200)
        _, uu = L.moments()
        rates.append(uu[0, 0, 0, :, 0] @ np.sin(2 * math.pi * y / n))
    assert abs(rates[1] / rates[0] - 1) < 5e-3


def test_streaming_direction_advects_downstream():
    """A transverse wave u_y = A sin(kx) on a uniform stream u_x = U is carried
    downstream: after t steps its phase is k (x - U t) (streaming moves f_i
    along +c_i, eq. streaming)."""
    n, U, amp, t = 32, 0.05, 1e-4, 64
    k = 2 * math.pi / n
    x = np.arange(n)
    u = np.zeros((3, 1, 1, 1, n))
    u[0] = U
    u[1, 0, 0, 0] = amp * np.sin(k * x)
    L = O.Lattice(n, 1, 1, tau=0.55)
    L.init(1.0, u)
    L.step(t)
    uy = L.moments()[1][1, 0, 0, 0]
    phase = math.atan2(uy @ np.cos(k * x), uy @ np.sin(k * x))  # uy ~ sin(kx + phase)
    assert abs(phase - (-k * U * t)) < 0.05 * k * U * t


def test_obstacle_channel_period_two_mode():
    """In a forced channel with a bounce-back sphere the flow settles into a
    steady field plus a non-decaying period-2 (staggered) oscillation: the
    single-step change u_t - u_{t-1} stalls at a finite level while the
    two-step change u_t - u_{t-2} keeps decaying.  This is why the steady-state
    residual of the warm-start study is measured over two steps."""
    wl = W.sphere_channels(1, nx=32, ny=16, nz=16, seed=5, rmin=3, rmax=4, nmin=1, nmax=1, fmin=1e-5, fmax=1e-5)
    solid = wl["solid"]
    F = np.zeros((3,) + solid.shape)
    F[0] = wl["fx"][0]
    L = O.Lattice(32, 16, 16, tau=0.8, wall=(0, 1, 0), solid=solid, force=F)
    L.init(np.ones(solid.shape), np.zeros((3,) + solid.shape))
    fl = ~solid.astype(bool)
    L.step(2500)
    u0 = L.moments()[1]
    L.step(1)
    u1 = L.moments()[1]
    L.step(1)
    u2 = L.moments()[1]
    n = np.linalg.norm(u2[:, fl])
    one = np.linalg.norm((u2 - u1)[:, fl]) / n
    two = np.linalg.norm((u2 - u0)[:, fl]) / (2 * n)
    assert one > 1e-7 and two < 1e-9, (one, two)


def test_four_rolls_mill_second_order():
    """Four-rolls mill (Sec. III; Re = 100, u0 = 1e-3, one node in z, a
    per-node force field): the oracle's steady velocity converges to the
    analytic Navier-Stokes steady state at second order, the paper's printed
    rate being 1.998.  Started from the analytic field (the steady state does
    not depend on the start; after two relaxation times of the box the error
    is within 3e-4 of its converged value)."""
    errs = {}
    for n in (8, 16):
        wl = W.four_rolls_mill(n)
        L = O.Lattice(n, n, 1, tau=wl["tau"], force=wl["force"])
        L.init(np.ones(wl["shape"]), wl["u_exact"])
        L.step(int(2 * wl["t_relax"]))
        u = L.moments()[1]
        errs[n] = np.linalg.norm(u[:2] - wl["u_exact"][:2]) / np.linalg.norm(wl["u_exact"][:2])
        assert abs(u[2]).max() < 1e-15  # the flow stays planar (to rounding)
    rate = math.log2(errs[8] / errs[16])
    assert 1.9 < rate < 2.1, (errs, rate)
    assert errs[16] < 0.03


# ---------------------------------------------------------------------------
# comparison models of Sec. III: truncated equilibrium (M5) and forcing (M4, M5)

def test_second_order_equilibrium_is_textbook_form():
    g = W.generator(31)
    for _ in range(5):
        rho, u = g.uniform(0.9, 1.1), g.uniform(-0.2, 0.2, 3)
        cu = C @ u
        ref = WGT * rho * (1 + cu / CS2 + cu ** 2 / (2 * CS2 ** 2) - (u @ u) / (2 * CS2))
        np.testing.assert_allclose(O.feq_order(rho, u, 2), ref, atol=1e-15)
        np.testing.assert_allclose(O.feq_order(rho, u, 6), O.feq(rho, u), atol=0)


def test_second_order_forcing_is_guo_form_and_printed_table():
    """H1 + H2 of eq. forcing is the Guo et al. forcing w_i [(c - u).F/cs2 +
    (c.u)(c.F)/cs4], and its central moments are the first truncation table of
    the forcing discussion in Sec. II, entry by entry (R0 and R4..R9 zero)."""
    g = W.generator(32)
    for _ in range(5):
        u, F = g.uniform(-0.2, 0.2, 3), g.uniform(-1e-2, 1e-2, 3)
        cu, cF = C @ u, C @ F
        guo = WGT * ((cF - u @ F) / CS2 + cu * cF / CS2 ** 2)
        f2 = O.forcing_order(u, F, 2)
        np.testing.assert_allclose(f2, guo, atol=1e-17)
        R = O.central_moments(u, f2)
        ux, uy, uz = u
        Fx, Fy, Fz = F
        cs2, cs4 = CS2, CS2 ** 2
        table = {
            1: Fx, 2: Fy, 3: Fz,
            10: 2 * Fx * cs2 - Fx * uy ** 2 - 2 * Fy * ux * uy - Fx * uz ** 2 - 2 * Fz * ux * uz,
            11: 2 * Fy * cs2 - Fy * ux ** 2 - 2 * Fx * uy * ux - Fy * uz ** 2 - 2 * Fz * uy * uz,
            12: 2 * Fz * cs2 - Fz * ux ** 2 - 2 * Fx * uz * ux - Fz * uy ** 2 - 2 * Fy * uz * uy,
            13: -Fx * uy ** 2 - 2 * Fy * ux * uy + Fx * uz ** 2 + 2 * Fz * ux * uz,
            14: -Fy * ux ** 2 - 2 * Fx * uy * ux + Fy * uz ** 2 + 2 * Fz * uy * uz,
            15: -Fz * ux ** 2 - 2 * Fx * uz * ux + Fz * uy ** 2 + 2 * Fy * uz * uy,
            16: -Fz * ux * uy - Fy * ux * uz - Fx * uy * uz,
            17: 4 * (Fy * ux ** 2 * uy + Fz * ux ** 2 * uz + Fx * ux * uy ** 2 + Fx * ux * uz ** 2
                     + Fz * uy ** 2 * uz + Fy * uy * uz ** 2),
            18: 4 * (Fy * ux ** 2 * uy + Fz * ux ** 2 * uz + Fx * ux * uy ** 2 + Fx * ux * uz ** 2
                     - Fz * uy ** 2 * uz - Fy * uy * uz ** 2),
            19: 4 * ux * (Fx * uy ** 2 + Fy * ux * uy - Fx * uz ** 2 - Fz * ux * uz),
            20: 2 * ux * (Fz * ux * uy + Fy * ux * uz + 2 * Fx * uy * uz),
            21: 2 * uy * (Fz * ux * uy + 2 * Fy * ux * uz + Fx * uy * uz),
            22: 2 * uz * (2 * Fz * ux * uy + Fy * ux * uz + Fx * uy * uz),
            23: Fx * cs4 - 3 * Fx * uy ** 2 * uz ** 2 - 6 * Fz * ux * uy ** 2 * uz - Fx * uy ** 2 / 3
                - 6 * Fy * ux * uy * uz ** 2 - 2 * Fy * ux * uy / 3 - Fx * uz ** 2 / 3 - 2 * Fz * ux * uz / 3,
            24: Fy * cs4 - 3 * Fy * ux ** 2 * uz ** 2 - 6 * Fz * uy * ux ** 2 * uz - Fy * ux ** 2 / 3
                - 6 * Fx * uy * ux * uz ** 2 - 2 * Fx * uy * ux / 3 - Fy * uz ** 2 / 3 - 2 * Fz * uy * uz / 3,
            25: Fz * cs4 - 3 * Fz * ux ** 2 * uy ** 2 - 6 * Fy * uz * ux ** 2 * uy - Fz * ux ** 2 / 3
                - 6 * Fx * uz * ux * uy ** 2 - 2 * Fx * uz * ux / 3 - Fz * uy ** 2 / 3 - 2 * Fy * uz * uy / 3,
            26: 8 * (Fz * ux ** 2 * uy ** 2 * uz + Fy * ux ** 2 * uy * uz ** 2 + Fx * ux * uy ** 2 * uz ** 2)
                + 4 * cs2 * (Fy * ux ** 2 * uy + Fz * ux ** 2 * uz + Fx * ux * uy ** 2 + Fx * ux * uz ** 2
                             + Fz * uy ** 2 * uz + Fy * uy * uz ** 2),
        }
        for j in range(27):
            assert abs(R[j] - table.get(j, 0.0)) < 1e-15, (j, R[j], table.get(j, 0.0))


@pytest.mark.parametrize("eq_order,force_order", [(6, 2), (2, 2), (2, 6)])
def test_comparison_models_conserve_mass_and_add_force(eq_order, force_order):
    g = W.generator(33)
    F = g.uniform(-1e-3, 1e-3, 3)
    for _ in range(5):
        f = W.random_populations((1,), seed=int(g.integers(1 << 30)))[:, 0]
        fs = O.collide_model(f, F, 1 / 0.7, eq_order, force_order)
        assert abs(fs.sum() - f.sum()) < 1e-15
        np.testing.assert_allclose(C.T @ fs - C.T @ f, F, atol=1e-15)
    # with the complete equilibrium and forcing the model route is the method itself
    np.testing.assert_allclose(O.collide_model(f, F, 1 / 0.7, 6, 6), O.collide_closed(f, F, 1 / 0.7), atol=2e-15)


@pytest.mark.parametrize("order", [2, 6])
def test_bgk_control_is_population_space_bgk(order):
    """Relaxing every central moment with omega is the population-space BGK
    collision f* = f - omega (f - f^eq) + (1 - omega / 2) F (T-bar is
    invertible), with the equilibrium and forcing of the given order."""
    g = W.generator(34)
    F = g.uniform(-1e-3, 1e-3, 3)
    omega = 1 / 0.62
    for _ in range(5):
        f = W.random_populations((1,), seed=int(g.integers(1 << 30)))[:, 0]
        rho = f.sum()
        u = (C.T @ f + F / 2) / rho
        ref = f - omega * (f - O.feq_order(rho, u, order)) + (1 - omega / 2) * O.forcing_order(u, F, order)
        np.testing.assert_allclose(O.collide_model(f, F, omega, order, order, bgk=True), ref, atol=2e-15)


# ---------------------------------------------------------------------------
# Shan-Chen pseudo-potential force of the static-droplet test (Sec. III)

def test_pseudopotential_force_properties():
    """Uniform density: no force.  Any density: the forces sum to zero (each
    pair interaction appears with both signs, Newton's third law).  Density
    varying along x only: the 27-velocity sum collapses to the 1D weights
    (1/6 for c_x = +-1), F_x = -G psi(x) (psi(x+1) - psi(x-1)) / 6 and
    F_y = F_z = 0."""
    G = -6.0
    assert np.abs(O.pseudopotential_force(np.full((1, 4, 5, 6), 0.7), G)).max() < 1e-15
    rho = W.generator(35).uniform(0.1, 2.0, size=(2, 5, 6, 7))
    F = O.pseudopotential_force(rho, G)
    assert np.abs(F.sum(axis=(1, 2, 3, 4))).max() < 1e-12
    x = np.arange(12)
    r1 = 1.0 + 0.5 * np.sin(2 * np.pi * x / 12) + 0.2 * np.cos(4 * np.pi * x / 12)
    rho = np.broadcast_to(r1, (1, 3, 4, 12)).copy()
    F = O.pseudopotential_force(rho, G)
    psi = 1 - np.exp(-r1)
    fx = -G * psi * (np.roll(psi, -1) - np.roll(psi, 1)) / 6
    np.testing.assert_allclose(F[0][0, 1, 2], fx, atol=1e-15)
    assert np.abs(F[1:]).max() < 1e-15
