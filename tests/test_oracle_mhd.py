"""Pins of the CPU oracle of the magnetic-field lattice (App. C) and of its
Lorentz-force coupling to the fluid (De Rosis, Huang & Coreixas, PRE 2019,
arXiv:1905.10182), against facts fixed by the paper and by mathematics."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import mhd as M

XI, WM = M.constants()
CSM2 = 0.25


def test_lattice_matches_printed_list():
    assert XI.T.tolist() == [[0, 1, -1, 0, 0, 0, 0], [0, 0, 0, 1, -1, 0, 0], [0, 0, 0, 0, 0, 1, -1]]
    np.testing.assert_allclose(WM, [0.25] + [0.125] * 6, atol=0)
    # quadrature: cs^2 = 1/4 for D3Q7
    assert abs(WM.sum() - 1) < 1e-16
    np.testing.assert_allclose(np.einsum("l,la,lb->ab", WM, XI, XI), CSM2 * np.eye(3), atol=1e-16)


def test_equilibrium_moments():
    """sum_l h^eq_l = b and sum_l xi_lb h^eq_la = u_b b_a - b_b u_a (the
    electric tensor of ideal MHD)."""
    g = W.generator(91)
    for _ in range(10):
        b, u = g.uniform(-0.2, 0.2, 3), g.uniform(-0.1, 0.1, 3)
        h = M.heq(b, u)
        np.testing.assert_allclose(h.sum(axis=0), b, atol=1e-16)
        np.testing.assert_allclose(np.einsum("lb,la->ba", XI, h), np.outer(u, b) - np.outer(b, u), atol=1e-17)


def diffusion_rate(n, tau_m, t1=100, t2=400):
    """Decay rate of b_y = B sin(2 pi x / n) at rest, in units of eta k^2."""
    L = M.MagneticLattice(n, 1, 1, tau_m)
    s = np.sin(2 * math.pi * np.arange(n) / n)
    b = np.zeros((3, 1, 1, n))
    b[1, 0, 0] = 1e-3 * s
    L.init(b)
    for _ in range(t1):
        L.step()
    a = L.fields()[0][1, 0, 0] @ s
    for _ in range(t2 - t1):
        L.step()
    c = L.fields()[0][1, 0, 0] @ s
    eta = (tau_m - 0.5) * CSM2
    return -math.log(c / a) / (t2 - t1) / (eta * (2 * math.pi / n) ** 2)


def test_resistivity_is_printed_relation():
    """eta = cs^2 (1/omega_m - 1/2) with cs^2 = 1/4: the decay rate of a
    magnetic shear wave tends to eta k^2 at second order."""
    for tau_m in (0.6, 0.9):
        e = [abs(diffusion_rate(n, tau_m) - 1) for n in (16, 32, 64)]
        assert e[2] < 2e-3
        assert 3.5 < e[0] / e[1] < 4.5 and 3.5 < e[1] / e[2] < 4.5, e


def test_uniform_flow_advects_the_field():
    """Induction with a uniform u: b(x, t) = b(x - u t) (plus diffusion), so
    the phase of b_y = B sin(kx) moves by -k U t."""
    n, U, t = 32, 0.05, 64
    k = 2 * math.pi / n
    x = np.arange(n)
    L = M.MagneticLattice(n, 1, 1, 0.55)
    b = np.zeros((3, 1, 1, n))
    b[1, 0, 0] = 1e-3 * np.sin(k * x)
    u = np.zeros((3, 1, 1, n))
    u[0] = U
    L.init(b, u)
    for _ in range(t):
        L.step(u)
    by = L.fields(u)[0][1, 0, 0]
    phase = math.atan2(by @ np.cos(k * x), by @ np.sin(k * x))
    assert abs(phase - (-k * U * t)) < 0.03 * k * U * t


def test_mean_field_is_conserved():
    g = W.generator(92)
    n = (6, 5, 4)
    L = M.MagneticLattice(*n[::-1], tau_m=0.7)
    b = g.uniform(-1e-2, 1e-2, (3,) + n)
    u = g.uniform(-0.05, 0.05, (3,) + n)
    L.init(b, u)
    for _ in range(10):
        L.step(u)
    np.testing.assert_allclose(L.fields()[0].sum(axis=(1, 2, 3)), b.sum(axis=(1, 2, 3)), atol=1e-15)


def test_population_current_tends_to_curl():
    """At rest the population current (reading C1) converges to the
    central-difference curl of b at second order; a wrong factor (for
    instance tau_m - 1/2 instead of tau_m) would leave a fixed ratio."""
    diffs = []
    for n in (16, 32, 64):
        L = M.MagneticLattice(n, n, 1, 0.8)
        k = 2 * math.pi / n
        X, Y = np.meshgrid(np.arange(n), np.arange(n))
        b = np.zeros((3, 1, n, n))
        b[0, 0] = -1e-3 * np.sin(k * Y)
        b[1, 0] = 1e-3 * np.sin(2 * k * X)
        L.init(b)
        for _ in range(20):
            L.step()
        _, jp = L.fields(current="populations")
        _, jf = L.fields(current="stencil")
        diffs.append(np.linalg.norm(jp - jf) / np.linalg.norm(jf))
    assert diffs[2] < 0.01
    assert 3.2 < diffs[0] / diffs[1] < 4.5 and 3.2 < diffs[1] / diffs[2] < 4.5, diffs


def test_lorentz_force_is_cross_product():
    g = W.generator(93)
    j, b = g.normal(size=(3, 2, 3, 4)), g.normal(size=(3, 2, 3, 4))
    F = M.lorentz(j, b)
    np.testing.assert_allclose(F, np.cross(j, b, axis=0), atol=1e-15)
    assert abs((F * b).sum(axis=0)).max() < 1e-14 and abs((F * j).sum(axis=0)).max() < 1e-14


def alfven_frequency_error(n, current, B0=0.05, tau=0.6, tau_m=0.6):
    """Standing Alfven wave on a uniform field B0 x: b_y = eps cos(kx), u = 0.
    Linear MHD with F = j x b gives modes exp(lambda t), lambda =
    -(nu + eta) k^2 / 2 +- i sqrt(k^2 B0^2 - ((nu - eta) k^2 / 2)^2); the
    measured zero-crossing spacing pi / omega against that omega."""
    eps, k = 1e-4, 2 * math.pi / n
    x = np.arange(n)
    b = np.zeros((3, 1, 1, n))
    b[0] = B0
    b[1, 0, 0] = eps * np.cos(k * x)
    S = M.MHD(n, 1, 1, tau, tau_m, current=current)
    S.init(np.ones((1, 1, n)), np.zeros((3, 1, 1, n)), b)
    nu, eta = (tau - 0.5) / 3, (tau_m - 0.5) * CSM2
    w = math.sqrt(k * k * B0 * B0 - ((nu - eta) * k * k / 2) ** 2)
    c = np.cos(k * x)
    ser = []
    for _ in range(int(2.2 * math.pi / w)):
        ser.append(S.mag.fields()[0][1, 0, 0] @ c)
        S.step()
    z = [i + ser[i] / (ser[i] - ser[i + 1]) for i in range(len(ser) - 1) if ser[i] * ser[i + 1] < 0]
    return math.pi / (z[1] - z[0]) / w - 1


def test_alfven_wave_speed_with_stencil_current():
    """The Lorentz force F = j x b on the D3Q27 fluid makes b_y, u_y an
    Alfven wave of speed B0 / sqrt(rho): with the central-difference current
    its frequency converges to k B0 at second order."""
    e = [alfven_frequency_error(n, "stencil") for n in (32, 64, 128)]
    assert abs(e[2]) < 5e-4
    assert 3.5 < e[0] / e[1] < 4.5 and 3.5 < e[1] / e[2] < 4.5, e


def test_alfven_wave_speed_with_population_current():
    """The population current omits the time derivative of the equilibrium
    electric tensor, which for a wave on B0 x is -2 B0^2 d_x b_y (first-order
    Chapman-Enskog), so j comes out as (1 - 2 B0^2/cs^2) curl b and the
    frequency as sqrt(1 - 2 B0^2/cs^2) k B0: about -1 % at B0 = 0.05 at every
    resolution."""
    B0 = 0.05
    expect = math.sqrt(1 - 2 * B0 * B0 / CSM2) - 1
    for n in (32, 64):
        assert abs(alfven_frequency_error(n, "populations", B0=B0) - expect) < 1.5e-3


def test_coupled_step_conserves_mass_and_mean_field():
    n = 12
    g = W.generator(94)
    u = 0.02 * g.uniform(-1, 1, (3, 1, n, n))
    u[2] = 0
    b = 0.02 * g.uniform(-1, 1, (3, 1, n, n))
    b[2] = 0
    S = M.MHD(n, n, 1, 0.7, 0.7)
    S.init(np.ones((1, n, n)), u, b)
    m0 = S.fluid.f.sum()
    S.step(20)
    rho, uu, bb, _ = S.state()
    assert abs(S.fluid.f.sum() / m0 - 1) < 1e-14
    np.testing.assert_allclose(bb.sum(axis=(1, 2, 3)), b.sum(axis=(1, 2, 3)), atol=1e-14)
    assert abs(uu[2]).max() < 1e-15 and abs(bb[2]).max() < 1e-15  # planar fields stay planar


# ---------------------------------------------------------------------------
# walls (reading C3) and the Hartmann flow (Sec. III)

def test_field_diffusion_between_walls():
    """With b = 0 imposed at walls halfway outside nodes 0 and n - 1, the
    mode sin(pi (y + 1/2) / n) decays at eta (pi / n)^2: the Dirichlet value
    sits at the half-way wall, to second order."""
    rates = []
    for n in (8, 16, 32):
        L = M.MagneticLattice(1, n, 1, 0.8, wall=(0, 1, 0))
        s = np.sin(math.pi * (np.arange(n) + 0.5) / n)
        b = np.zeros((3, 1, n, 1))
        b[0, 0, :, 0] = 1e-3 * s
        L.init(b)
        for _ in range(50):
            L.step()
        a = L.fields()[0][0, 0, :, 0] @ s
        for _ in range(200):
            L.step()
        c = L.fields()[0][0, 0, :, 0] @ s
        eta = 0.3 * CSM2
        rates.append(-math.log(c / a) / 200 / (eta * (math.pi / n) ** 2) - 1)
    assert abs(rates[2]) < 5e-3
    assert 3.5 < rates[0] / rates[1] < 4.5 and 3.5 < rates[1] / rates[2] < 4.5, rates


def test_wall_value_is_reached_at_steady_state():
    # a uniform field equal to the wall value is a steady state at rest
    n = 10
    bw = np.array([0.01, -0.02, 0.005])
    L = M.MagneticLattice(1, n, 1, 0.7, wall=(0, 1, 0), b_wall=bw)
    L.init(np.broadcast_to(bw.reshape(3, 1, 1, 1), (3, 1, n, 1)))
    for _ in range(20):
        L.step()
    np.testing.assert_allclose(L.fields()[0][:, 0, :, 0], np.broadcast_to(bw[:, None], (3, n)), atol=1e-16)


def hartmann_error(L, Ha, current, nu=0.1, umax=1e-3, relax=4.0):
    """Relative L2 error of the steady Hartmann profile in a channel of width
    L (walls at y = -1/2 and L - 1/2, the field (0, B0, 0) imposed there,
    eta = nu, driven by a uniform force G).  With b_x = 0 at both walls the
    one-dimensional MHD equations give
    u(s) = G a^2 / (nu Ha tanh Ha) [1 - cosh(Ha s / a) / cosh Ha],
    a = L / 2, Ha = B0 a / sqrt(nu eta) (the Hartmann number as the paper
    defines it, B0 L / sqrt(4 rho nu eta))."""
    a = L / 2.0
    B0 = Ha * nu / a
    G = umax * nu * Ha * math.tanh(Ha) / (a * a)
    S = M.MHD(1, L, 1, 0.5 + 3 * nu, 0.5 + 4 * nu, current=current, wall=(0, 1, 0), b_wall=(0.0, B0, 0.0))
    b = np.zeros((3, 1, L, 1))
    b[1] = B0
    S.init(np.ones((1, L, 1)), np.zeros((3, 1, L, 1)), b)
    S.body_force = (G, 0.0, 0.0)
    S.step(int(relax * a * a / nu))
    u = S.state()[1][0, 0, :, 0]
    s = np.arange(L) - (L - 1) / 2.0
    ua = G * a * a / (nu * Ha * math.tanh(Ha)) * (1 - np.cosh(Ha * s / a) / math.cosh(Ha))
    return float(np.linalg.norm(u - ua) / np.linalg.norm(ua))


@pytest.mark.parametrize("current", ["populations", "stencil"])
def test_hartmann_profile_converges(current):
    """Hartmann flow (Sec. III) at Ha = 3: the steady velocity converges to the
    analytic profile, at second order for the population current and close to
    it for the stencil current (whose ghost value at the wall is one-sided)."""
    e = [hartmann_error(L, 3.0, current) for L in (8, 16, 32)]
    rates = [math.log2(e[k] / e[k + 1]) for k in range(2)]
    assert e[2] < (5e-3 if current == "populations" else 1e-2), e
    lo = 1.8 if current == "populations" else 1.5
    assert all(r > lo for r in rates), (e, rates)
