"""Pins of the FP64 CPU oracle of the two-dimensional D2Q9 model (App. B of
De Rosis, Huang & Coreixas, PRE 2019, arXiv:1905.10182) against facts fixed by
the paper and by mathematics, not against the oracle itself.

Printed tables live in tests/golden/d2q9_tables.json with their citations.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import d2q9 as D

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "d2q9_tables.json")))
CS2 = 1.0 / 3.0
CX, CY, WGT, OPP = D.constants()
C = np.stack([CX, CY], axis=1).astype(float)


def table_vector(entries, rho=None, F=None, k=None, omega=None):
    out = np.zeros(9)
    for j, (kind, comp, coef, p) in entries.items():
        if kind == "rho":
            x = rho
        elif kind == "F":
            x = F[comp]
        else:
            x = (1.0 - omega) * k[comp]
        out[int(j)] = coef * x * CS2 ** p
    return out


def phi(c, u):
    """1D factor of the complete equilibrium on {-1, 0, 1}: the unique
    weights with moments 1, u, cs^2 + u^2."""
    return 2.0 / 3.0 - u * u if c == 0 else (CS2 + u * u + c * u) / 2.0


def product_feq(rho, u):
    return np.array([rho * phi(CX[i], u[0]) * phi(CY[i], u[1]) for i in range(9)])


@pytest.fixture(scope="module")
def cells():
    rho, u = W.random_cells(20, seed=71, umax=0.2)
    return [(r, v[:2]) for r, v in zip(rho, u)]


def rand_pops(seed):
    return W.random_populations((), seed=seed, q=9).ravel()


# ---------------------------------------------------------------------------
# lattice

def test_lattice_matches_printed_list():
    g = GOLD["lattice"]
    assert list(CX) == g["cx"] and list(CY) == g["cy"]
    np.testing.assert_allclose(WGT, [eval(w) for w in g["w"]], rtol=0, atol=1e-17)
    for i in range(9):
        assert np.all(C[OPP[i]] == -C[i])


def test_weights_quadrature_moments():
    assert abs(WGT.sum() - 1) < 1e-15
    np.testing.assert_allclose(WGT @ C, 0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", WGT, C, C), CS2 * np.eye(2), atol=1e-16)
    assert abs(np.sum(WGT * C[:, 0] ** 2 * C[:, 1] ** 2) - CS2 ** 2) < 1e-16


# ---------------------------------------------------------------------------
# equilibrium (eq. eq:D2Q9)

def test_complete_equilibrium_is_tensor_product(cells):
    for rho, u in cells:
        np.testing.assert_allclose(D.feq_order(rho, u, 4), product_feq(rho, u), rtol=1e-14, atol=1e-16)


def test_second_order_equilibrium_is_textbook_form(cells):
    for rho, u in cells:
        cu = C @ u
        ref = WGT * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * (u @ u))
        np.testing.assert_allclose(D.feq_order(rho, u, 2), ref, atol=1e-15)


def test_equilibrium_central_moments_are_printed_table(cells):
    for rho, u in cells:
        k = D.central_moments(u, D.feq_order(rho, u, 4))
        np.testing.assert_allclose(k, table_vector(GOLD["equilibrium"]["entries"], rho=rho), atol=1e-15)


def test_second_order_equilibrium_is_not_galilean_invariant():
    rho, u = 1.0, np.array([0.1, -0.05])
    k = D.central_moments(u, D.feq_order(rho, u, 2))
    # the fourth-order moment k8 picks up rho ux^2 uy^2-type terms
    assert abs(k[8] - rho * CS2 ** 2) > 1e-5


# ---------------------------------------------------------------------------
# forcing (App. B)

def test_forcing_is_velocity_gradient_of_equilibrium(cells):
    """The complete Hermite forcing term is F . grad_u f^eq at rho = 1,
    checked by central differences of the independent product form."""
    g = W.generator(72)
    h = 1e-5
    for _, u in cells:
        F = g.uniform(-1, 1, 2)
        num = np.zeros(9)
        for a in range(2):
            e = np.zeros(2)
            e[a] = h
            num += F[a] * (product_feq(1.0, u + e) - product_feq(1.0, u - e)) / (2 * h)
        np.testing.assert_allclose(D.forcing_order(u, F, 4), num, atol=1e-10)


def test_forcing_central_moments_are_printed_table(cells):
    g = W.generator(73)
    for _, u in cells:
        F = g.uniform(-1e-2, 1e-2, 2)
        R = D.central_moments(u, D.forcing_order(u, F, 4))
        np.testing.assert_allclose(R, table_vector(GOLD["forcing"]["entries"], F=F), atol=1e-17)


def test_second_order_forcing_is_guo_form(cells):
    """Keeping H1 + H2 gives the Guo et al. term w_i [(c - u).F/cs^2 + (c.u)(c.F)/cs^4]."""
    g = W.generator(74)
    for _, u in cells:
        F = g.uniform(-1e-2, 1e-2, 2)
        guo = WGT * (((C - u) @ F) / CS2 + (C @ u) * (C @ F) / CS2 ** 2)
        np.testing.assert_allclose(D.forcing_order(u, F, 2), guo, atol=1e-17)


# ---------------------------------------------------------------------------
# basis and its inverse (eq. system2)

def test_basis_determinant_is_velocity_free():
    """T-bar(u) is T-bar(0) times a unit-triangular binomial shift, so its
    determinant does not depend on u.  |det| = 128: the monomial basis
    (1, c, c^2) x (1, c, c^2) is the tensor product of two 3 x 3 Vandermonde
    matrices of det 2 (det 2^3 * 2^3 = 64), and the pair (k3, k4) =
    (K20 + K02, K20 - K02) contributes a factor 2."""
    d0 = np.linalg.det(D.basis(np.zeros(2)))
    g = W.generator(75)
    for _ in range(10):
        u = g.uniform(-0.3, 0.3, 2)
        assert abs(np.linalg.det(D.basis(u)) - d0) < 1e-12 * abs(d0)
    assert abs(abs(d0) - 128.0) < 1e-11


def test_literal_reconstruction_inverts_the_transform():
    g = W.generator(76)
    for _ in range(20):
        u = g.uniform(-0.3, 0.3, 2)
        f = g.normal(size=9)
        np.testing.assert_allclose(D.reconstruct_literal(u, D.central_moments(u, f)), f, atol=1e-13)


# ---------------------------------------------------------------------------
# collision

def test_collide_literal_equals_closed_form():
    g = W.generator(77)
    for _ in range(30):
        f = rand_pops(int(g.integers(1 << 30)))
        F = g.uniform(-1e-2, 1e-2, 2)
        omega = g.uniform(0.5, 1.95)
        np.testing.assert_allclose(D.collide_closed(f, F, omega), D.collide_model(f, F, omega), atol=2e-15)


def test_post_collision_moments_are_printed_table():
    g = W.generator(78)
    for _ in range(10):
        f = rand_pops(int(g.integers(1 << 30)))
        F = g.uniform(-1e-2, 1e-2, 2)
        omega = g.uniform(0.5, 1.95)
        rho, u = D.macroscopic(f, F)
        k = D.central_moments(u, f)
        ks = D.central_moments(u, D.collide_closed(f, F, omega))
        expect = table_vector(GOLD["post_collision_forced"]["entries"], rho=rho, F=F, k=k, omega=omega)
        np.testing.assert_allclose(ks, expect, atol=2e-15)
        np.testing.assert_allclose(D.post_collision(rho, k[4], k[5], F, omega), expect, atol=1e-16)


def test_relaxation_matrix_is_printed_diagonal():
    """The general relaxation k* = (I - L) k + L k^eq + (I - L/2) R with the
    printed L (omega on k4, k5 only) reproduces the literal collision."""
    g = W.generator(79)
    L_on = GOLD["relaxation"]["omega_on"]
    for _ in range(5):
        f = rand_pops(int(g.integers(1 << 30)))
        F = g.uniform(-1e-2, 1e-2, 2)
        omega = g.uniform(0.5, 1.95)
        rho, u = D.macroscopic(f, F)
        L = np.array([omega if j in L_on else 1.0 for j in range(9)])
        k = D.central_moments(u, f)
        keq = table_vector(GOLD["equilibrium"]["entries"], rho=rho)
        R = table_vector(GOLD["forcing"]["entries"], F=F)
        ks = (1 - L) * k + L * keq + (1 - L / 2) * R
        np.testing.assert_allclose(np.linalg.solve(D.basis(u).T, ks), D.collide_model(f, F, omega), atol=2e-15)


def test_pre_collision_first_moments_are_minus_half_force():
    f = rand_pops(80)
    F = np.array([3e-3, -1e-3])
    rho, u = D.macroscopic(f, F)
    np.testing.assert_allclose(D.central_moments(u, f)[1:3], -F / 2, atol=1e-16)


def test_mass_and_momentum_with_half_force():
    g = W.generator(81)
    for _ in range(20):
        f = rand_pops(int(g.integers(1 << 30)))
        F = g.uniform(-1e-2, 1e-2, 2)
        fs = D.collide_closed(f, F, g.uniform(0.5, 1.95))
        assert abs(fs.sum() - f.sum()) < 1e-15
        np.testing.assert_allclose(fs @ C, f @ C + F, atol=1e-16)


def test_equilibrium_is_fixed_point_without_force(cells):
    for rho, u in cells:
        fe = product_feq(rho, u)
        for omega in (0.6, 1.0, 1.7):
            np.testing.assert_allclose(D.collide_closed(fe, np.zeros(2), omega), fe, atol=1e-15)


def test_omega_one_reduces_to_equilibrium_plus_half_forcing():
    g = W.generator(82)
    for _ in range(10):
        f = rand_pops(int(g.integers(1 << 30)))
        F = g.uniform(-1e-2, 1e-2, 2)
        rho, u = D.macroscopic(f, F)
        np.testing.assert_allclose(D.collide_closed(f, F, 1.0), product_feq(rho, u) + 0.5 * D.forcing_order(u, F),
                                   atol=1e-15)


def test_shear_moment_relaxes_with_omega():
    # the perturbation d_i = w_i cx cy at rest has k5 as its only central moment
    f = product_feq(1.0, np.zeros(2))
    d = WGT * C[:, 0] * C[:, 1] * 1e-3
    k = D.central_moments(np.zeros(2), d)
    assert abs(k[5]) > 1e-5 and np.abs(np.delete(k, 5)).max() < 1e-18
    omega = 1.3
    np.testing.assert_allclose(D.collide_closed(f + d, np.zeros(2), omega) - f, (1 - omega) * d, atol=2e-16)


def test_bulk_moment_is_equilibrated():
    # the isotropic perturbation d_i = w_i (|c|^2 - 2 cs^2) at rest carries only
    # k3 (and k8), which the relaxation matrix sets to equilibrium in one step
    f = product_feq(1.0, np.zeros(2))
    d = WGT * ((C ** 2).sum(axis=1) - 2 * CS2) * 1e-3
    k = D.central_moments(np.zeros(2), d)
    assert abs(k[3]) > 1e-5 and abs(k[0]) < 1e-18
    np.testing.assert_allclose(D.collide_closed(f + d, np.zeros(2), 0.7), f, atol=2e-16)


# ---------------------------------------------------------------------------
# lattice level

def test_literal_and_closed_lattices_agree():
    g = W.generator(83)
    f0 = W.random_populations((5, 7), seed=84, q=9)
    force = g.uniform(-1e-3, 1e-3, (2, 5, 7))
    A = D.Lattice2D(7, 5, tau=0.7, force=force)
    B = D.Lattice2D(7, 5, tau=0.7, force=force)
    A.load_populations(f0)
    B.load_populations(f0)
    A.step(5, "literal")
    B.step(5, "closed")
    np.testing.assert_allclose(A.f, B.f, atol=1e-14)


def test_periodic_mass_momentum_bookkeeping():
    g = W.generator(85)
    f0 = W.random_populations((6, 5), seed=86, q=9)
    force = g.uniform(-1e-3, 1e-3, (2, 6, 5))
    L = D.Lattice2D(5, 6, tau=0.9, force=force)
    L.load_populations(f0)
    m0 = L.f.sum()
    p0 = L.f.reshape(9, -1).sum(axis=1) @ C
    L.step(10)
    assert abs(L.f.sum() / m0 - 1) < 1e-14
    np.testing.assert_allclose(L.f.reshape(9, -1).sum(axis=1) @ C, p0 + 10 * force.sum(axis=(1, 2)), atol=1e-13)


def test_streaming_moves_populations_along_their_velocity():
    # a single population on one cell, collision-free in this check: after one
    # step of the closed route at rest the mass that left along c_i sits at x + c_i
    n = 5
    L = D.Lattice2D(n, n, tau=1.0)
    L.init(1.0, np.zeros((2, n, n)))
    f_before = L.f.copy()
    L.step(1)
    np.testing.assert_allclose(L.f, f_before, atol=1e-16)  # rest state is a fixed point
    u = np.zeros((2, n, n))
    u[0, 2, 2] = 0.1
    L.init(1.0, u)
    L.step(1)
    rho, _ = L.moments()
    # with omega = 1 the momentum-carrying excess of cell (2, 2) moved to x = 3
    assert rho[2, 3] > rho[2, 1]


def shear_wave_rate_2d(n, tau, amp=1e-4, t1=100, t2=400):
    y = np.arange(n)
    s = np.sin(2 * math.pi * y / n)
    u = np.zeros((2, n, 1))
    u[0, :, 0] = amp * s
    L = D.Lattice2D(1, n, tau=tau)
    L.init(1.0, u)
    L.step(t1)
    a = L.moments()[1][0, :, 0] @ s
    L.step(t2 - t1)
    b = L.moments()[1][0, :, 0] @ s
    nu = (tau - 0.5) / 3
    return -math.log(b / a) / (t2 - t1) / (nu * (2 * math.pi / n) ** 2)


def test_shear_wave_viscosity():
    """nu = (tau - 1/2) cs^2: the shear-wave decay rate tends to nu k^2 at
    second order in the resolution."""
    for tau in (0.6, 0.8):
        e = [abs(shear_wave_rate_2d(n, tau) - 1) for n in (16, 32, 64)]
        assert e[2] < 1e-3
        assert 3.5 < e[0] / e[1] < 4.5 and 3.5 < e[1] / e[2] < 4.5, e


def test_four_rolls_mill_second_order():
    """Four-rolls mill (Sec. III, Re = 100, u0 = 1e-3) on the D2Q9 model: the
    steady velocity converges to the analytic steady state at second order
    (the paper prints a rate of 1.998).  Started from the analytic field and
    run for two relaxation times of the box."""
    errs = {}
    for n in (8, 16):
        wl = W.four_rolls_mill_2d(n)
        L = D.Lattice2D(n, n, tau=wl["tau"], force=wl["force"])
        L.init(np.ones(wl["shape"]), wl["u_exact"])
        L.step(int(2 * wl["t_relax"]))
        u = L.moments()[1]
        errs[n] = np.linalg.norm(u - wl["u_exact"]) / np.linalg.norm(wl["u_exact"])
    rate = math.log2(errs[8] / errs[16])
    assert 1.9 < rate < 2.1, (errs, rate)
    assert errs[16] < 0.03
