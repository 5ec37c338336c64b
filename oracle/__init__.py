"""FP64 CPU oracle of the D3Q27 central-moment LBM with Hermite forcing.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
cpu_baseline leg of bench.py, never by the product package.  It shares no code
with the HIP path.  The arithmetic lives in ``cmlbm_oracle.c`` (plain C, FP64,
unshifted populations); this module only marshals numpy arrays through ctypes.

Paper: De Rosis, Huang & Coreixas, Phys. Rev. E (2019), arXiv:1905.10182,
Sec. II (method) -- see the header of cmlbm_oracle.c for the equation map and
the readings taken where the paper is silent.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_libs = {}

_dpp = ctypes.POINTER(ctypes.c_double)
_ldp = ctypes.POINTER(ctypes.c_longdouble)
_dp = _dpp
_ip = ctypes.POINTER(ctypes.c_int)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def _load(extended=False):
    if extended not in _libs:
        path = _build.build(force=False, extended=extended)
        lib = ctypes.CDLL(path)
        _dp = _ldp if extended else _dpp
        _real = ctypes.c_longdouble if extended else ctypes.c_double
        lib.orc_lattice_constants.argtypes = [_ip, _ip, _ip, _dp, _ip]
        lib.orc_feq.argtypes = [_real, _dp, _dp]
        lib.orc_forcing.argtypes = [_dp, _dp, _dp]
        lib.orc_feq_order.argtypes = [_real, _dp, ctypes.c_int, _dp]
        lib.orc_forcing_order.argtypes = [_dp, _dp, ctypes.c_int, _dp]
        lib.orc_collide_model.argtypes = [_dp, _dp, _real, ctypes.c_int, ctypes.c_int, _dp]
        lib.orc_collide_model.restype = ctypes.c_int
        lib.orc_collide_model_bgk.argtypes = [_dp, _dp, _real, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp]
        lib.orc_collide_model_bgk.restype = ctypes.c_int
        lib.orc_basis.argtypes = [_dp, _dp]
        lib.orc_central_moments.argtypes = [_dp, _dp, _dp]
        lib.orc_macroscopic.argtypes = [_dp, _dp, _dp, _dp]
        lib.orc_reconstruct_literal.argtypes = [_dp, _dp, _dp]
        lib.orc_reconstruct_literal.restype = ctypes.c_int
        lib.orc_reconstruct_fast.argtypes = [_dp, _dp, _dp]
        lib.orc_collide_literal.argtypes = [_dp, _dp, _real, _dp]
        lib.orc_collide_literal.restype = ctypes.c_int
        lib.orc_collide_closed.argtypes = [_dp, _dp, _real, _dp]
        lib.orc_pre_collision.argtypes = [_dp, _dp, _dp]
        lib.orc_post_collision.argtypes = [_real, _dp, _dp, _real, _dp]
        lib.orc_lattice_init.argtypes = [ctypes.c_int] * 4 + [_u8p, _dp, _dp, _dp]
        lib.orc_lattice_step.argtypes = [ctypes.c_int] * 4 + [_ip, _u8p, _dp, _real,
                                                              ctypes.c_int, ctypes.c_int, _dp, _dp]
        lib.orc_lattice_step.restype = ctypes.c_int
        lib.orc_lattice_moments.argtypes = [ctypes.c_int] * 4 + [_u8p, _dp, _dp, _dp, _dp]
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_pseudopotential_force.argtypes = [ctypes.c_int] * 4 + [_real, _dp, _dp]
        lib.orc_collide_cells.argtypes = [ctypes.c_long, _dp, _dp, _real, ctypes.c_int, _dp]
        lib.orc_collide_cells.restype = ctypes.c_int
        _libs[extended] = lib
    return _libs[extended]


def _d(a):
    if a.dtype == np.longdouble and np.longdouble != np.float64:
        return a.ctypes.data_as(_ldp)
    return a.ctypes.data_as(_dpp)


def _vec(x, n):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(n))
    return a


def num_threads():
    return _load().orc_num_threads()


def constants():
    """(cx, cy, cz, w, opp) of the D3Q27 lattice in the paper's order."""
    lib = _load()
    cx = np.zeros(27, np.int32)
    cy = np.zeros(27, np.int32)
    cz = np.zeros(27, np.int32)
    w = np.zeros(27)
    opp = np.zeros(27, np.int32)
    ip = lambda a: a.ctypes.data_as(_ip)  # noqa: E731
    lib.orc_lattice_constants(ip(cx), ip(cy), ip(cz), _d(w), ip(opp))
    return cx, cy, cz, w, opp


def feq(rho, u):
    """Complete 27-Hermite equilibrium (eq. eq:truncation)."""
    out = np.zeros(27)
    _load().orc_feq(float(rho), _d(_vec(u, 3)), _d(out))
    return out


def forcing(u, F):
    """Complete Hermite forcing term (eq. forcing), F a force density."""
    out = np.zeros(27)
    _load().orc_forcing(_d(_vec(u, 3)), _d(_vec(F, 3)), _d(out))
    return out


def feq_order(rho, u, order):
    """Equilibrium of eq. eq:truncation keeping Hermite tensors up to `order` (2 or 6)."""
    out = np.zeros(27)
    _load().orc_feq_order(float(rho), _d(_vec(u, 3)), int(order), _d(out))
    return out


def forcing_order(u, F, order):
    """Forcing term of eq. forcing keeping Hermite tensors up to `order` (2 = Guo, 6 = complete)."""
    out = np.zeros(27)
    _load().orc_forcing_order(_d(_vec(u, 3)), _d(_vec(F, 3)), int(order), _d(out))
    return out


def pseudopotential_force(rho, G, extended=False):
    """Shan-Chen force -G psi(x) sum_i w_i c_i psi(x + c_i), psi = 1 - exp(-rho), periodic;
    rho (nb, nz, ny, nx) -> F (3, nb, nz, ny, nx)."""
    dt = np.longdouble if extended else np.float64
    rho = np.ascontiguousarray(np.asarray(rho, dt))
    nb, nz, ny, nx = rho.shape
    F = np.zeros((3,) + rho.shape, dt)
    _load(extended).orc_pseudopotential_force(nx, ny, nz, nb, dt(G), _d(rho), _d(F))
    return F


def collide_model(f, F, omega, eq_order, force_order, bgk=False):
    """Literal collision with a truncated equilibrium / forcing (the comparison models of Sec. III);
    bgk=True relaxes every central moment with omega (single-relaxation-time control)."""
    out = np.zeros(27)
    if _load().orc_collide_model_bgk(_d(_vec(f, 27)), _d(_vec(F, 3)), float(omega), int(eq_order),
                                     int(force_order), int(bool(bgk)), _d(out)) != 0:
        raise ArithmeticError("singular central-moment matrix")
    return out


def basis(u):
    """Transformation matrix T-bar with T[i, j] = T_j(c_i - u) (eq. basis)."""
    out = np.zeros((27, 27))
    _load().orc_basis(_d(_vec(u, 3)), _d(out))
    return out


def central_moments(u, f):
    """k = T-bar^T f."""
    out = np.zeros(27)
    _load().orc_central_moments(_d(_vec(u, 3)), _d(_vec(f, 27)), _d(out))
    return out


def macroscopic(f, F=(0.0, 0.0, 0.0)):
    """rho and the half-force-corrected u (eq. macroscopic)."""
    rho = np.zeros(1)
    u = np.zeros(3)
    _load().orc_macroscopic(_d(_vec(f, 27)), _d(_vec(F, 3)), _d(rho), _d(u))
    return float(rho[0]), u


def reconstruct_literal(u, k):
    out = np.zeros(27)
    if _load().orc_reconstruct_literal(_d(_vec(u, 3)), _d(_vec(k, 27)), _d(out)) != 0:
        raise ArithmeticError("singular central-moment matrix")
    return out


def reconstruct_fast(u, k):
    out = np.zeros(27)
    _load().orc_reconstruct_fast(_d(_vec(u, 3)), _d(_vec(k, 27)), _d(out))
    return out


def pre_collision(f, u):
    """k_4..k_8 of eq. pre_collision."""
    out = np.zeros(5)
    _load().orc_pre_collision(_d(_vec(f, 27)), _d(_vec(u, 3)), _d(out))
    return out


def post_collision(rho, k48, F, omega):
    """Basis-ordered post-collision central moments (eq. post_collision_central_moments_forcing)."""
    out = np.zeros(27)
    _load().orc_post_collision(float(rho), _d(_vec(k48, 5)), _d(_vec(F, 3)), float(omega), _d(out))
    return out


def collide_literal(f, F, omega):
    out = np.zeros(27)
    if _load().orc_collide_literal(_d(_vec(f, 27)), _d(_vec(F, 3)), float(omega), _d(out)) != 0:
        raise ArithmeticError("singular central-moment matrix")
    return out


def collide_closed(f, F, omega):
    out = np.zeros(27)
    _load().orc_collide_closed(_d(_vec(f, 27)), _d(_vec(F, 3)), float(omega), _d(out))
    return out


def collide_cells(f, F, omega, variant="closed", extended=False):
    """Collide independent cells: f (27, n), F (3, n) or None -> f* (27, n)."""
    dt = np.longdouble if extended else np.float64
    f = np.ascontiguousarray(np.asarray(f, dt))
    n = f.shape[1]
    Fp = None
    if F is not None:
        F = np.ascontiguousarray(np.broadcast_to(np.asarray(F, dt), (3, n)))
        Fp = _d(F)
    out = np.zeros_like(f)
    rc = _load(extended).orc_collide_cells(n, _d(f), Fp, omega, Lattice.VARIANTS[variant], _d(out))
    if rc != 0:
        raise ArithmeticError("singular central-moment matrix")
    return out


class Lattice:
    """A lattice of nb independent nx*ny*nz boxes advanced by the oracle.

    State ``f`` is the pre-collision population array f(x, t), shape
    (27, nb, nz, ny, nx), unshifted FP64, paper order.  ``wall`` gives per axis
    (x, y, z) 0 = periodic or 1 = halfway bounce-back walls; ``solid`` is an
    optional (nb, nz, ny, nx) mask; ``force`` an optional (3, nb, nz, ny, nx)
    force-density field (constant in time).  ``extended=True`` runs the same
    oracle in 80-bit long double (arrays np.longdouble).
    """

    # closed form and literal route of the method (M1); literal routes of the
    # comparison models M4 (second-order forcing), M5 (second-order equilibrium
    # and forcing), a second-order equilibrium with the complete forcing, and
    # the single-relaxation-time (BGK) controls with the second-order or the
    # complete equilibrium and forcing
    VARIANTS = {"closed": 0, "literal": 1, "m4": 2, "m5": 3, "eq2": 4, "bgk": 5, "bgk6": 6}

    def __init__(self, nx, ny, nz, nb=1, tau=0.8, wall=(0, 0, 0), solid=None, force=None, extended=False):
        self.extended = bool(extended)
        self.dtype = np.longdouble if self.extended else np.float64
        self.lib = _load(self.extended)
        self.nx, self.ny, self.nz, self.nb = int(nx), int(ny), int(nz), int(nb)
        self.shape = (self.nb, self.nz, self.ny, self.nx)
        self.N = int(np.prod(self.shape))
        if tau <= 0.5:
            raise ValueError("tau must exceed 1/2")
        self.tau = float(tau)
        self.omega = 1 / self.dtype(self.tau)
        self.wall = np.ascontiguousarray(np.asarray(wall, np.int32).reshape(3))
        self.solid = None if solid is None else np.ascontiguousarray(
            np.asarray(solid).reshape(self.shape).astype(np.uint8))
        self.set_force(force)
        self.f = np.zeros((27,) + self.shape, self.dtype)
        self._tmp = np.zeros_like(self.f)
        self.t = 0

    def set_force(self, force):
        if force is None:
            self.force = None
        else:
            self.force = np.ascontiguousarray(
                np.broadcast_to(np.asarray(force, self.dtype), (3,) + self.shape).copy())

    def _solid_p(self):
        return None if self.solid is None else self.solid.ctypes.data_as(_u8p)

    def _force_p(self):
        return None if self.force is None else _d(self.force)

    def init(self, rho, u):
        rho = np.ascontiguousarray(np.broadcast_to(np.asarray(rho, self.dtype), self.shape))
        u = np.ascontiguousarray(np.broadcast_to(np.asarray(u, self.dtype), (3,) + self.shape))
        self.lib.orc_lattice_init(self.nx, self.ny, self.nz, self.nb, self._solid_p(), _d(rho), _d(u),
                                 _d(self.f))
        self.t = 0

    def load_populations(self, f):
        self.f[...] = np.asarray(f, self.dtype).reshape(self.f.shape)

    def step(self, nsteps=1, variant="closed"):
        rc = self.lib.orc_lattice_step(self.nx, self.ny, self.nz, self.nb, self.wall.ctypes.data_as(_ip),
                                      self._solid_p(), self._force_p(), self.omega,
                                      self.VARIANTS[variant], int(nsteps), _d(self.f), _d(self._tmp))
        if rc != 0:
            raise ArithmeticError("singular central-moment matrix during a literal step")
        self.t += int(nsteps)

    def moments(self):
        """(rho, u) at the current time; solid cells report 0."""
        rho = np.zeros(self.shape, self.dtype)
        u = np.zeros((3,) + self.shape, self.dtype)
        self.lib.orc_lattice_moments(self.nx, self.ny, self.nz, self.nb, self._solid_p(), self._force_p(),
                                    _d(self.f), _d(rho), _d(u))
        return rho, u

    def reductions(self, u_snapshot=None):
        """Global monitors of the current state (time t, force in effect):
        the module-level reductions() of moments()."""
        rho, u = self.moments()
        return reductions(rho, u, self.solid, self.force, u_snapshot)


# ---------------------------------------------------------------------------
# global monitors of a lattice state

def reductions(rho, u, solid=None, force=None, u_snapshot=None):
    """Global sums over the fluid cells of each batch member, from the
    macroscopic fields of eq. macroscopic (rho, and the half-force-corrected
    u, as Lattice.moments() returns them).

    rho (nb, ...), u (3, nb, ...), solid (nb, ...) or None, force (3, nb, ...)
    or None (the force density in effect), u_snapshot (3, nb, ...) or None.
    Returns one dict per member:
      mass      sum rho                                   (eq. macroscopic)
      mom       sum_x sum_i f_i c_i = sum (rho u - F/2)   (eq. macroscopic: rho u = sum f c + F/2)
      ke        sum rho |u|^2 / 2   (the kinetic energy whose mean is the
                stability monitor of the Orszag-Tang and static-droplet tests, Sec. III)
      umax      max |u|
      u2        sum |u|^2
      du2       sum |u - u_snapshot|^2 (0 without a snapshot)
      residual  sqrt(du2 / u2): the relative L2 norm of eq. error applied to
                two velocity fields (0 without a snapshot)
      fluid     number of fluid cells
      nonfinite number of fluid cells whose rho or u is not finite
    Sums are taken in the arrays' precision (FP64, or 80-bit for the
    extended oracle)."""
    rho = np.asarray(rho)
    u = np.asarray(u)
    nb = rho.shape[0]
    fl = np.ones(rho.shape, bool) if solid is None else ~np.asarray(solid, bool).reshape(rho.shape)
    out = []
    for b in range(nb):
        m = fl[b]
        r = rho[b][m]
        ub = u[:, b][:, m]
        fin = np.isfinite(r) & np.isfinite(ub).all(axis=0)
        mom = (r * ub).sum(axis=1)
        if force is not None:
            mom = mom - np.asarray(force, u.dtype)[:, b][:, m].sum(axis=1) / 2
        usq = (ub * ub).sum(axis=0)
        d = {"mass": r.sum(), "mom": mom, "ke": (r * usq).sum() / 2, "umax": np.sqrt(usq.max()) if usq.size else 0.0,
             "u2": usq.sum(), "du2": 0.0, "residual": 0.0, "fluid": int(m.sum()), "nonfinite": int((~fin).sum())}
        if u_snapshot is not None:
            dv = ub - np.asarray(u_snapshot, u.dtype)[:, b][:, m]
            d["du2"] = (dv * dv).sum()
            d["residual"] = np.sqrt(d["du2"] / d["u2"])
        out.append(d)
    return out
