"""FP64 CPU oracle of the two-dimensional D2Q9 central-moment model with
Hermite forcing (App. B of De Rosis, Huang & Coreixas, Phys. Rev. E 2019,
arXiv:1905.10182).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
cpu_baseline leg of bench.py, never by the product package.  The arithmetic
lives in ``d2q9_oracle.c`` (plain C, FP64, unshifted populations, compiled into
the same liboracle.so as the D3Q27 oracle); this module marshals numpy arrays
through ctypes.  See the header of d2q9_oracle.c for the readings taken.
"""
import ctypes

import numpy as np

from . import _load as _load_lib, _d, _ip, _vec

Q = 9
_ready = {}


def _load(extended=False):
    lib = _load_lib(extended)
    if extended not in _ready:
        dp = ctypes.POINTER(ctypes.c_longdouble) if extended else ctypes.POINTER(ctypes.c_double)
        real = ctypes.c_longdouble if extended else ctypes.c_double
        ci = ctypes.c_int
        lib.orc2_lattice_constants.argtypes = [_ip, _ip, dp, _ip]
        lib.orc2_feq_order.argtypes = [real, dp, ci, dp]
        lib.orc2_forcing_order.argtypes = [dp, dp, ci, dp]
        lib.orc2_basis.argtypes = [dp, dp]
        lib.orc2_central_moments.argtypes = [dp, dp, dp]
        lib.orc2_macroscopic.argtypes = [dp, dp, dp, dp]
        lib.orc2_reconstruct_literal.argtypes = [dp, dp, dp]
        lib.orc2_reconstruct_literal.restype = ci
        lib.orc2_collide_model.argtypes = [dp, dp, real, ci, ci, dp]
        lib.orc2_collide_model.restype = ci
        lib.orc2_post_collision.argtypes = [real, real, real, dp, real, dp]
        lib.orc2_collide_closed.argtypes = [dp, dp, real, dp]
        lib.orc2_collide_cells.argtypes = [ctypes.c_long, dp, dp, real, ci, dp]
        lib.orc2_collide_cells.restype = ci
        lib.orc2_lattice_init.argtypes = [ci, ci, dp, dp, dp]
        lib.orc2_lattice_step.argtypes = [ci, ci, dp, real, ci, ci, dp, dp]
        lib.orc2_lattice_step.restype = ci
        lib.orc2_lattice_moments.argtypes = [ci, ci, dp, dp, dp, dp]
        _ready[extended] = True
    return lib


def constants():
    """(cx, cy, w, opp) of the D2Q9 lattice in the order of App. B."""
    cx = np.zeros(Q, np.int32)
    cy = np.zeros(Q, np.int32)
    w = np.zeros(Q)
    opp = np.zeros(Q, np.int32)
    ip = lambda a: a.ctypes.data_as(_ip)  # noqa: E731
    _load().orc2_lattice_constants(ip(cx), ip(cy), _d(w), ip(opp))
    return cx, cy, w, opp


def feq_order(rho, u, order=4):
    """Equilibrium of eq. eq:D2Q9 up to Hermite order `order` (2 or 4)."""
    out = np.zeros(Q)
    _load().orc2_feq_order(float(rho), _d(_vec(u, 2)), int(order), _d(out))
    return out


def forcing_order(u, F, order=4):
    """Hermite forcing term of App. B up to order `order` (2 = Guo, 4 = complete)."""
    out = np.zeros(Q)
    _load().orc2_forcing_order(_d(_vec(u, 2)), _d(_vec(F, 2)), int(order), _d(out))
    return out


def basis(u):
    """T[i, j] = T-bar_j(c_i - u) of App. B."""
    out = np.zeros((Q, Q))
    _load().orc2_basis(_d(_vec(u, 2)), _d(out))
    return out


def central_moments(u, f):
    out = np.zeros(Q)
    _load().orc2_central_moments(_d(_vec(u, 2)), _d(_vec(f, Q)), _d(out))
    return out


def macroscopic(f, F=(0.0, 0.0)):
    rho = np.zeros(1)
    u = np.zeros(2)
    _load().orc2_macroscopic(_d(_vec(f, Q)), _d(_vec(F, 2)), _d(rho), _d(u))
    return float(rho[0]), u


def reconstruct_literal(u, k):
    out = np.zeros(Q)
    if _load().orc2_reconstruct_literal(_d(_vec(u, 2)), _d(_vec(k, Q)), _d(out)) != 0:
        raise ArithmeticError("singular central-moment matrix")
    return out


def post_collision(rho, k4, k5, F, omega):
    """The printed post-collision central moments of App. B."""
    out = np.zeros(Q)
    _load().orc2_post_collision(float(rho), float(k4), float(k5), _d(_vec(F, 2)), float(omega), _d(out))
    return out


def collide_model(f, F, omega, eq_order=4, force_order=4):
    out = np.zeros(Q)
    if _load().orc2_collide_model(_d(_vec(f, Q)), _d(_vec(F, 2)), float(omega), int(eq_order),
                                  int(force_order), _d(out)) != 0:
        raise ArithmeticError("singular central-moment matrix")
    return out


def collide_closed(f, F, omega):
    out = np.zeros(Q)
    _load().orc2_collide_closed(_d(_vec(f, Q)), _d(_vec(F, 2)), float(omega), _d(out))
    return out


def collide_cells(f, F, omega, variant="closed", extended=False):
    """Collide independent cells: f (9, n), F (2, n) or None -> f* (9, n)."""
    dt = np.longdouble if extended else np.float64
    f = np.ascontiguousarray(np.asarray(f, dt))
    n = f.shape[1]
    Fp = None
    if F is not None:
        F = np.ascontiguousarray(np.broadcast_to(np.asarray(F, dt), (2, n)))
        Fp = _d(F)
    out = np.zeros_like(f)
    if _load(extended).orc2_collide_cells(n, _d(f), Fp, omega, Lattice2D.VARIANTS[variant], _d(out)) != 0:
        raise ArithmeticError("singular central-moment matrix")
    return out


class Lattice2D:
    """A periodic nx * ny D2Q9 lattice advanced by the oracle.

    State ``f`` is the pre-collision population array f(x, t), shape
    (9, ny, nx), unshifted FP64, App. B order; ``force`` an optional (2, ny, nx)
    force-density field (constant in time).
    """

    # closed form and literal route of the method; literal routes with the Guo
    # (second-order) forcing, with second-order equilibrium and forcing, and
    # with a second-order equilibrium and the complete forcing
    VARIANTS = {"closed": 0, "literal": 1, "m4": 2, "m5": 3, "eq2": 4}

    def __init__(self, nx, ny, tau=0.8, force=None, extended=False):
        self.extended = bool(extended)
        self.dtype = np.longdouble if self.extended else np.float64
        self.lib = _load(self.extended)
        self.nx, self.ny = int(nx), int(ny)
        self.shape = (self.ny, self.nx)
        if tau <= 0.5:
            raise ValueError("tau must exceed 1/2")
        self.tau = float(tau)
        self.omega = 1 / self.dtype(self.tau)
        self.set_force(force)
        self.f = np.zeros((Q,) + self.shape, self.dtype)
        self._tmp = np.zeros_like(self.f)
        self.t = 0

    def set_force(self, force):
        self.force = None if force is None else np.ascontiguousarray(
            np.broadcast_to(np.asarray(force, self.dtype), (2,) + self.shape).copy())

    def _force_p(self):
        return None if self.force is None else _d(self.force)

    def init(self, rho, u):
        rho = np.ascontiguousarray(np.broadcast_to(np.asarray(rho, self.dtype), self.shape))
        u = np.ascontiguousarray(np.broadcast_to(np.asarray(u, self.dtype), (2,) + self.shape))
        self.lib.orc2_lattice_init(self.nx, self.ny, _d(rho), _d(u), _d(self.f))
        self.t = 0

    def load_populations(self, f):
        self.f[...] = np.asarray(f, self.dtype).reshape(self.f.shape)

    def step(self, nsteps=1, variant="closed"):
        rc = self.lib.orc2_lattice_step(self.nx, self.ny, self._force_p(), self.omega, self.VARIANTS[variant],
                                        int(nsteps), _d(self.f), _d(self._tmp))
        if rc != 0:
            raise ArithmeticError("singular central-moment matrix during a literal step")
        self.t += int(nsteps)

    def moments(self):
        """(rho (ny, nx), u (2, ny, nx)) at the current time."""
        rho = np.zeros(self.shape, self.dtype)
        u = np.zeros((2,) + self.shape, self.dtype)
        self.lib.orc2_lattice_moments(self.nx, self.ny, self._force_p(), _d(self.f), _d(rho), _d(u))
        return rho, u
