"""FP64 CPU oracle of the magnetic-field lattice of App. C (D3Q7 vector
populations, BGK) and of its coupling to the D3Q27 fluid through the Lorentz
force F = j x b (De Rosis, Huang & Coreixas, Phys. Rev. E 2019,
arXiv:1905.10182, Sec. III and App. C).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
cpu_baseline leg of bench.py, never by the product package.  The arithmetic
lives in ``mhd_oracle.c`` (and, for the fluid, ``cmlbm_oracle.c``); this
module marshals numpy arrays and sequences one coupled step.  See the header
of mhd_oracle.c for the readings taken.
"""
import ctypes

import numpy as np

from . import Lattice, _d, _ip, _load as _load_lib

Q = 7
_ready = {}


def _load(extended=False):
    lib = _load_lib(extended)
    if extended not in _ready:
        dp = ctypes.POINTER(ctypes.c_longdouble) if extended else ctypes.POINTER(ctypes.c_double)
        real = ctypes.c_longdouble if extended else ctypes.c_double
        ci = ctypes.c_int
        lib.orc_mhd_constants.argtypes = [_ip, dp]
        lib.orc_mhd_heq.argtypes = [dp, dp, dp]
        lib.orc_mhd_init.argtypes = [ci, ci, ci, dp, dp, dp]
        lib.orc_mhd_step.argtypes = [ci, ci, ci, dp, real, dp, dp]
        lib.orc_mhd_step_walls.argtypes = [ci, ci, ci, _ip, dp, dp, real, dp, dp]
        lib.orc_curl_fd_walls.argtypes = [ci, ci, ci, _ip, dp, dp, dp]
        lib.orc_mhd_fields.argtypes = [ci, ci, ci, dp, real, dp, dp, dp]
        lib.orc_curl_fd.argtypes = [ci, ci, ci, dp, dp]
        lib.orc_lorentz.argtypes = [ctypes.c_long, dp, dp, dp]
        _ready[extended] = True
    return lib


def constants():
    """(xi (7, 3), w (7,)) of the D3Q7 set in the order of App. C."""
    xi = np.zeros((Q, 3), np.int32)
    w = np.zeros(Q)
    _load().orc_mhd_constants(xi.ctypes.data_as(_ip), _d(w))
    return xi, w


def heq(b, u):
    """Equilibrium of App. C for one cell: array (7, 3)."""
    out = np.zeros((Q, 3))
    _load().orc_mhd_heq(_d(np.ascontiguousarray(b, np.float64)), _d(np.ascontiguousarray(u, np.float64)),
                        _d(out))
    return out


def curl_fd(b, wall=None, b_wall=None):
    """Central-difference curl of b (3, nz, ny, nx): periodic axes, or the
    ghost value 2 b_wall - b beyond the walls flagged in `wall` (x, y, z)."""
    b = np.ascontiguousarray(b, np.float64)
    nz, ny, nx = b.shape[1:]
    j = np.zeros_like(b)
    if wall is None:
        _load().orc_curl_fd(nx, ny, nz, _d(b), _d(j))
    else:
        w = np.ascontiguousarray(wall, np.int32)
        bw = np.ascontiguousarray(np.zeros(3) if b_wall is None else b_wall, np.float64)
        _load().orc_curl_fd_walls(nx, ny, nz, w.ctypes.data_as(_ip), _d(bw), _d(b), _d(j))
    return j


def lorentz(j, b):
    j = np.ascontiguousarray(j, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    F = np.zeros_like(b)
    _load().orc_lorentz(b[0].size, _d(j), _d(b), _d(F))
    return F


class MagneticLattice:
    """The D3Q7 magnetic lattice alone on an nx * ny * nz box: periodic axes,
    or walls halfway between nodes on the axes flagged in `wall` (x, y, z)
    where b takes the value b_wall (reading C6).  State h (7, 3, nz, ny, nx);
    tau_m the magnetic relaxation time, eta = (tau_m - 1/2) / 4."""

    def __init__(self, nx, ny, nz, tau_m, extended=False, wall=(0, 0, 0), b_wall=(0.0, 0.0, 0.0)):
        self.extended = bool(extended)
        self.dtype = np.longdouble if self.extended else np.float64
        self.lib = _load(self.extended)
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.shape = (self.nz, self.ny, self.nx)
        if tau_m <= 0.5:
            raise ValueError("tau_m must exceed 1/2")
        self.tau_m = self.dtype(tau_m)
        self.h = np.zeros((Q, 3) + self.shape, self.dtype)
        self._tmp = np.zeros_like(self.h)
        self.wall = np.ascontiguousarray(wall, np.int32)
        self.b_wall = np.ascontiguousarray(b_wall, self.dtype)

    def _vec(self, v):
        return None if v is None else np.ascontiguousarray(np.broadcast_to(np.asarray(v, self.dtype),
                                                                           (3,) + self.shape))

    def init(self, b, u=None):
        b, u = self._vec(b), self._vec(u)
        self.lib.orc_mhd_init(self.nx, self.ny, self.nz, _d(b), None if u is None else _d(u), _d(self.h))

    def step(self, u=None):
        u = self._vec(u)
        self.lib.orc_mhd_step_walls(self.nx, self.ny, self.nz, self.wall.ctypes.data_as(_ip), _d(self.b_wall),
                                    None if u is None else _d(u), 1 / self.tau_m, _d(self.h), _d(self._tmp))

    def fields(self, u=None, current="populations"):
        """(b, j), each (3, nz, ny, nx); the current from the populations
        (reading C1) or by central differences of b ('stencil')."""
        u = self._vec(u)
        b = np.zeros((3,) + self.shape, self.dtype)
        j = np.zeros_like(b)
        self.lib.orc_mhd_fields(self.nx, self.ny, self.nz, None if u is None else _d(u), self.tau_m, _d(self.h),
                                _d(b), _d(j) if current == "populations" else None)
        if current != "populations":
            j = curl_fd(b.astype(np.float64), self.wall, self.b_wall.astype(np.float64)).astype(self.dtype)
        return b, j


class MHD:
    """Fluid (D3Q27 oracle, `variant` as in oracle.Lattice) coupled to the
    magnetic lattice through the Lorentz force, one box (nbatch = 1).  With
    `wall` both lattices have walls on the flagged axes (fluid: halfway
    bounce-back; field: b = b_wall there).  `body_force` (3 values, set after
    construction) is added to the Lorentz force (the driving of the Hartmann
    channel).

    One step:
      (a) u_lag = fluid velocity with the force in effect (the previous step's);
      (b) b and j from the magnetic populations (j with u_lag), F = j x b,
          set as the fluid force;
      (c) u = fluid velocity with F;
      (d) magnetic collision towards h^eq(b, u) and streaming;
      (e) fluid collision with F and streaming.
    """

    def __init__(self, nx, ny, nz, tau, tau_m, variant="closed", current="populations", extended=False,
                 wall=(0, 0, 0), b_wall=(0.0, 0.0, 0.0)):
        self.fluid = Lattice(nx, ny, nz, tau=tau, wall=wall, extended=extended)
        self.mag = MagneticLattice(nx, ny, nz, tau_m, extended=extended, wall=wall, b_wall=b_wall)
        self.body_force = None
        self.variant, self.current = variant, current
        self.shape = (nz, ny, nx)
        self.t = 0

    def init(self, rho, u, b):
        self.fluid.init(rho, np.asarray(u).reshape((3, 1) + self.shape))
        self.fluid.set_force(None)
        self.mag.init(b, u)
        self.t = 0

    def velocity(self):
        return self.fluid.moments()[1].reshape((3,) + self.shape)

    def step(self, n=1):
        for _ in range(int(n)):
            u_lag = self.velocity()
            b, j = self.mag.fields(u_lag, self.current)
            F = lorentz(j.astype(np.float64), b.astype(np.float64))
            if self.body_force is not None:
                F = F + np.asarray(self.body_force, np.float64).reshape(3, 1, 1, 1)
            self.fluid.set_force(F.reshape((3, 1) + self.shape))
            u = self.velocity()
            self.mag.step(u)
            self.fluid.step(1, self.variant)
            self.t += 1

    def state(self):
        """(rho, u, b, j) at the current time, the current with the force in effect."""
        rho, u = self.fluid.moments()
        u = u.reshape((3,) + self.shape)
        b, j = self.mag.fields(u, self.current)
        return rho.reshape(self.shape), u, b, j
