"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module holds workload definitions only -- initial density and velocity
fields, force densities, geometries and random draws -- and none of the
method's arithmetic.  Random numbers come from numpy's PCG64 with explicit
seeds, so every caller sees identical inputs.

Workloads (sizes as used by the tests and the benchmark):
  poiseuille      body-force channel, periodic x and z, bounce-back walls in y
  taylor_green    3D Taylor-Green vortex in a periodic cube
  kolmogorov      sinusoidally forced periodic cube
  sphere_channels batch of forced channels with spherical obstacles
"""
import math

import numpy as np


def generator(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def poiseuille(nx=32, ny=16, nz=16, tau=0.8, fx=1e-6, steps=1000):
    """Body-force Poiseuille channel 32x16x16: fluid at rest, rho = 1, uniform
    force density (fx, 0, 0), walls at y = -1/2 and y = ny - 1/2."""
    shape = (1, nz, ny, nx)
    return dict(name=f"poiseuille_{nx}x{ny}x{nz}", shape=shape, tau=tau, rho0=1.0, wall=(0, 1, 0),
                rho=np.ones(shape), u=np.zeros((3,) + shape), force=np.array([fx, 0.0, 0.0]), steps=steps)


def taylor_green_viscosity(n, u0=0.05, re=1600.0):
    """nu from Re = u0 (n / 2 pi) / nu (length scale 1/k)."""
    return u0 * n / (2.0 * math.pi * re)


def taylor_green(n, u0=0.05, re=1600.0, noise=1e-6, seed=1, rho0=1.0, steps=2000, dtype=np.float64):
    """3D Taylor-Green vortex on an n^3 periodic box.

    u = u0 (sin kx cos ky cos kz, -cos kx sin ky cos kz, 0), k = 2 pi / n,
    rho = rho0 + 3 rho0 u0^2/16 (cos 2kx + cos 2ky)(cos 2kz + 2) + U(-noise, noise)
    (the pressure field of the incompressible vortex divided by c_s^2 = 1/3),
    tau = 3 nu + 1/2 with nu fixed by Re."""
    nu = taylor_green_viscosity(n, u0, re)
    tau = 3.0 * nu + 0.5
    k = 2.0 * math.pi / n
    c = np.arange(n, dtype=np.float64) * k
    sx, cx_ = np.sin(c), np.cos(c)
    c2 = np.cos(2 * c)
    shape = (1, n, n, n)  # (b, z, y, x)
    ux = u0 * (cx_[None, :, None] * sx[None, None, :]) * cx_[:, None, None]
    uy = -u0 * (sx[None, :, None] * cx_[None, None, :]) * cx_[:, None, None]
    u = np.zeros((3,) + shape, dtype=dtype)
    u[0, 0] = ux
    u[1, 0] = uy
    rho = np.empty(shape, dtype=dtype)
    rho[0] = rho0 + 3.0 * rho0 * u0 * u0 / 16.0 * (c2[None, None, :] + c2[None, :, None]) * (c2[:, None, None] + 2.0)
    if noise:
        rho[0] += generator(seed).uniform(-noise, noise, size=(n, n, n))
    return dict(name=f"taylor_green_{n}", shape=shape, tau=tau, nu=nu, rho0=rho0, wall=(0, 0, 0), rho=rho, u=u,
                force=None, steps=steps, u0=u0)


def kolmogorov(n, f0=1e-5, tau=0.5005, kf=4, noise=1e-4, seed=2, steps=5000):
    """Kolmogorov flow on an n^3 periodic box: force density
    F_x(y) = f0 sin(2 pi kf y / n) on integer node rows y, rho = 1, velocity
    components i.i.d. U(-noise, noise)."""
    shape = (1, n, n, n)
    y = np.arange(n, dtype=np.float64)
    prof = np.zeros((n, 3))
    prof[:, 0] = f0 * np.sin(2.0 * math.pi * kf * y / n)
    u = generator(seed).uniform(-noise, noise, size=(3,) + shape)
    return dict(name=f"kolmogorov_{n}", shape=shape, tau=tau, rho0=1.0, wall=(0, 0, 0), rho=np.ones(shape), u=u,
                force_profile_y=prof, steps=steps)


def four_rolls_mill(n, u0=1e-3, re=100.0):
    """Two-dimensional four-rolls mill (Sec. III): an n x n periodic box, one
    node in z, driven by the body-force density
    F = 2 nu u0 psi^2 [sin(psi x) sin(psi y), cos(psi x) cos(psi y)], psi = 2 pi / n,
    on the integer node coordinates, with Re = u0 n / nu.  Its steady state is
    u = u0 [sin(psi x) sin(psi y), cos(psi x) cos(psi y)] (returned as u_exact,
    z component zero).  Arrays have the batch shape (1, 1, n, n)."""
    nu = u0 * n / re
    psi = 2.0 * math.pi / n
    c = np.arange(n, dtype=np.float64)
    sx, cx = np.sin(psi * c)[None, :], np.cos(psi * c)[None, :]  # varies along x (last axis)
    sy, cy = np.sin(psi * c)[:, None], np.cos(psi * c)[:, None]  # varies along y
    shape = (1, 1, n, n)
    u = np.zeros((3,) + shape)
    u[0] = (u0 * sx * sy).reshape(shape)
    u[1] = (u0 * cx * cy).reshape(shape)
    force = 2.0 * nu * psi * psi * u
    return dict(name=f"four_rolls_mill_{n}", shape=shape, tau=0.5 + 3.0 * nu, nu=nu, u0=u0, re=re, rho0=1.0,
                wall=(0, 0, 0), force=force, u_exact=u,
                # slowest relaxation time of the box (wavenumber psi): 1 / (nu psi^2)
                t_relax=1.0 / (nu * psi * psi))


def four_rolls_mill_2d(n, u0=1e-3, re=100.0, dtype=np.float64):
    """The four-rolls mill above on a genuinely two-dimensional n x n lattice
    (the D2Q9 model of App. B): the same force density and steady state with
    the z axis dropped.  Arrays have the shape (ny, nx) = (n, n), vectors
    (2, n, n), in `dtype` (float32 halves the host memory at large n)."""
    nu = u0 * n / re
    psi = 2.0 * math.pi / n
    c = np.arange(n, dtype=np.float64)
    s, co = np.sin(psi * c), np.cos(psi * c)
    u = np.empty((2, n, n), dtype)
    u[0] = u0 * np.outer(s, s)    # sin(psi x) sin(psi y), rows are y
    u[1] = u0 * np.outer(co, co)  # cos(psi x) cos(psi y)
    force = (2.0 * nu * psi * psi) * u
    return dict(name=f"four_rolls_mill_2d_{n}", shape=(n, n), tau=0.5 + 3.0 * nu, nu=nu, u0=u0, re=re, rho0=1.0,
                force=force, u_exact=u, t_relax=1.0 / (nu * psi * psi))


def static_droplet(n=200, radius=40.0, rho_in=1.0, rho_out=0.125, g=-6.0, tau=2.0, width=8.0):
    """Static droplet of the pseudo-potential test (Sec. III): a periodic n^3 box,
    a sphere of radius `radius` about the box centre at density rho_in in a
    vapour at rho_out = rho_in / 8, at rest; Shan-Chen interaction strength g.
    The paper states neither the radius, the relaxation time nor the interface
    profile; this workload uses radius n / 5, tau = 2 and a tanh interface
    rho(r) = (rho_in + rho_out) / 2 - (rho_in - rho_out) / 2 tanh(2 (r - R) / width)
    (width = 0: a sharp step, cells with r <= R inside)."""
    c = (np.arange(n) - (n - 1) / 2.0) ** 2
    r = np.sqrt(c[:, None, None] + c[None, :, None] + c[None, None, :])
    if width > 0:
        rho = 0.5 * (rho_in + rho_out) - 0.5 * (rho_in - rho_out) * np.tanh(2.0 * (r - radius) / width)
    else:
        rho = np.where(r <= radius, rho_in, rho_out)
    rho = rho[None].astype(np.float64)
    shape = (1, n, n, n)
    return dict(name=f"static_droplet_{n}_r{radius:g}", shape=shape, tau=tau, rho0=1.0, wall=(0, 0, 0), rho=rho,
                u=np.zeros((3,) + shape), g=g, radius=radius)


def sphere_channels(nb, nx=64, ny=32, nz=32, seed=1000, rmin=3.0, rmax=8.0, nmin=1, nmax=4, fmin=1e-6, fmax=1e-5,
                    tau=0.8):
    """Batch of nb forced channels (periodic x, z; walls in y) with 1-4 solid
    spheres each.  Radius U[rmin, rmax]; centre x, z uniform, y uniform in
    [r, ny - 1 - r]; node (x, y, z) is solid if its periodic distance (in x and
    z) to a centre is <= r.  Force density (F_x, 0, 0), F_x ~ U[fmin, fmax].
    Member b uses the seed seed + b, so members are reproducible one by one."""
    solid = np.zeros((nb, nz, ny, nx), np.uint8)
    fx = np.zeros(nb)
    spheres = []
    X = np.arange(nx)[None, None, :]
    Y = np.arange(ny)[None, :, None]
    Z = np.arange(nz)[:, None, None]
    for b in range(nb):
        g = generator(seed + b)
        ns = int(g.integers(nmin, nmax + 1))
        fx[b] = g.uniform(fmin, fmax)
        lst = []
        for _ in range(ns):
            r = g.uniform(rmin, rmax)
            cx = g.uniform(0, nx)
            cy = g.uniform(r, ny - 1 - r)
            cz = g.uniform(0, nz)
            dx = np.abs(X - cx)
            dx = np.minimum(dx, nx - dx)
            dz = np.abs(Z - cz)
            dz = np.minimum(dz, nz - dz)
            solid[b] |= ((dx * dx + (Y - cy) ** 2 + dz * dz) <= r * r).astype(np.uint8)
            lst.append((cx, cy, cz, r))
        spheres.append(lst)
    return dict(name=f"sphere_channels_{nb}x{nx}x{ny}x{nz}", shape=(nb, nz, ny, nx), tau=tau, rho0=1.0,
                wall=(0, 1, 0), solid=solid, fx=fx, spheres=spheres)


def random_populations(shape, seed, lo=0.8, hi=1.2, q=27):
    """Positive populations f_i = U(lo, hi) / q, array (q,) + shape: an
    arbitrary (non-equilibrium) pre-collision state for parity tests (q = 27
    for D3Q27, 9 for D2Q9)."""
    return generator(seed).uniform(lo, hi, size=(q,) + tuple(shape)) / float(q)


def representable(x, storage):
    """x (FP64 array) moved to a nearby value that the storage format holds
    exactly, so that both sides of a parity test start from the same numbers:
    FP64 unchanged; FP32 rounded to float32; FP16 as the solver stores it
    (256 x rounded to binary16, divided by 256); BF16 x in float32 with the
    low 16 bits cleared (truncated to an 8-bit significand).  Input
    preparation only."""
    x = np.asarray(x, np.float64)
    if storage == "fp64":
        return x.copy()
    if storage == "fp32":
        return x.astype(np.float32).astype(np.float64)
    if storage == "fp16":
        return (x * 256.0).astype(np.float16).astype(np.float64) / 256.0
    if storage == "bf16":
        b = np.ascontiguousarray(x.astype(np.float32)).view(np.uint32) & np.uint32(0xFFFF0000)
        return b.view(np.float32).astype(np.float64)
    raise ValueError(storage)


def random_cells(n, seed, umax=0.1, rho_lo=0.9, rho_hi=1.1):
    """n random (rho, u) pairs: rho ~ U[rho_lo, rho_hi], u_a ~ U[-umax, umax]."""
    g = generator(seed)
    return g.uniform(rho_lo, rho_hi, size=n), g.uniform(-umax, umax, size=(n, 3))
