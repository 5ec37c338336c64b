"""Python binding of libcmlbm_mhd (C ABI in include/cmlbm_mhd.h): the
magnetic-field lattice of App. C (D3Q7 vector populations) and the Lorentz
force F = j x b that couples it to the D3Q27 fluid solver.

Argument marshalling and step sequencing only: every arithmetic step runs in
the HIP kernels of libcmlbm_mhd.so and libcmlbm.so.  If a library is missing
this module raises; there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcmlbm_mhd.so")

OK, EINVAL, ENOMEM, EHIP, ESTATE = 0, -1, -2, -3, -5
FP64, FP32 = 0, 1
STORAGE = {"fp64": FP64, "fp32": FP32}
PERIODIC, WALL = 0, 1
CURRENT = {"populations": 0, "stencil": 1}

# Every entry point declared in include/cmlbm_mhd.h.
EXPORTS = ["cmlbm_mhd_required_bytes", "cmlbm_mhd_create", "cmlbm_mhd_set_wall_field", "cmlbm_mhd_set_body_force",
           "cmlbm_mhd_init", "cmlbm_mhd_fields", "cmlbm_mhd_step", "cmlbm_mhd_populations",
           "cmlbm_mhd_load_populations", "cmlbm_mhd_get_time", "cmlbm_mhd_destroy", "cmlbm_mhd_last_error",
           "cmlbm_mhd_status_string"]


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("tau_m", ctypes.c_double),
                ("storage", ctypes.c_int32), ("wall", ctypes.c_int32 * 3), ("flags", ctypes.c_uint32)]


class MhdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_status_string(code)}: {msg}")
        self.code = code


_lib = None


def load_library():
    """Load libcmlbm_mhd.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is missing: build it with `python -m paper_1905_10182_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    P = ctypes.POINTER(Params)
    lib.cmlbm_mhd_required_bytes.argtypes = [P, ctypes.POINTER(sz)]
    lib.cmlbm_mhd_create.argtypes = [P, vp, sz, vp, sz, ctypes.POINTER(vp)]
    lib.cmlbm_mhd_set_wall_field.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.cmlbm_mhd_set_body_force.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.cmlbm_mhd_init.argtypes = [vp, vp, vp, vp]
    lib.cmlbm_mhd_fields.argtypes = [vp, vp, ctypes.c_int, vp, vp, vp, vp]
    lib.cmlbm_mhd_step.argtypes = [vp, vp, vp]
    lib.cmlbm_mhd_populations.argtypes = [vp, vp, vp]
    lib.cmlbm_mhd_load_populations.argtypes = [vp, vp, vp]
    lib.cmlbm_mhd_get_time.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.cmlbm_mhd_destroy.argtypes = [vp]
    lib.cmlbm_mhd_last_error.argtypes = [vp]
    lib.cmlbm_mhd_last_error.restype = ctypes.c_char_p
    lib.cmlbm_mhd_status_string.argtypes = [ctypes.c_int]
    lib.cmlbm_mhd_status_string.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("cmlbm_mhd_last_error", "cmlbm_mhd_status_string"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _status_string(code):
    try:
        return load_library().cmlbm_mhd_status_string(code).decode()
    except OSError:
        return str(code)


def make_params(nx, ny, nz, tau_m=0.8, storage="fp64", wall=(0, 0, 0), flags=0):
    p = Params()
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    p.tau_m = float(tau_m)
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    for a in range(3):
        p.wall[a] = int(wall[a])
    p.flags = int(flags)
    return p


def _host3(v):
    a = (ctypes.c_double * 3)(*[float(x) for x in np.asarray(v, np.float64).ravel()])
    return a


def required_bytes(params):
    n = ctypes.c_size_t()
    rc = load_library().cmlbm_mhd_required_bytes(ctypes.byref(params), ctypes.byref(n))
    if rc != OK:
        raise MhdError(rc, "invalid lattice parameters")
    return n.value


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class MagneticLattice:
    """One magnetic-lattice handle over torch-allocated device buffers.
    Vector fields are (3, nz, ny, nx) tensors of the storage dtype.  `wall`
    flags axes (x, y, z) with walls, where b takes the value b_wall."""

    def __init__(self, nx, ny, nz, tau_m, storage="fp64", device="cuda", wall=(0, 0, 0), b_wall=None):
        import torch

        self.torch = torch
        self.lib = load_library()
        self.params = make_params(nx, ny, nz, tau_m, storage, wall)
        self.shape = (int(nz), int(ny), int(nx))
        self.dtype = torch.float64 if self.params.storage == FP64 else torch.float32
        self.device = torch.device(device)
        self.pop_bytes = required_bytes(self.params)
        self._a = torch.empty(self.pop_bytes, dtype=torch.uint8, device=self.device)
        self._b = torch.empty(self.pop_bytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        rc = self.lib.cmlbm_mhd_create(ctypes.byref(self.params), _ptr(self._a), self.pop_bytes, _ptr(self._b),
                                       self.pop_bytes, ctypes.byref(h))
        if rc != OK:
            raise MhdError(rc, "cmlbm_mhd_create failed")
        self.handle = h
        if b_wall is not None:
            self.set_wall_field(b_wall)

    def set_wall_field(self, b_wall):
        self._check(self.lib.cmlbm_mhd_set_wall_field(self.handle, _host3(b_wall)), "set_wall_field")

    def set_body_force(self, f0):
        """Uniform force density added to the Lorentz force that fields() writes."""
        self._check(self.lib.cmlbm_mhd_set_body_force(self.handle, _host3(f0)), "set_body_force")

    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _check(self, rc, what):
        if rc != OK:
            raise MhdError(rc, f"{what}: {self.lib.cmlbm_mhd_last_error(self.handle).decode()}")

    def _vec(self, v):
        """A (3, nz, ny, nx) contiguous device tensor of the storage dtype (the
        same object if it already is one)."""
        if v is None:
            return None
        if isinstance(v, np.ndarray) and not v.flags.writeable:
            v = np.array(v)
        t = self.torch.as_tensor(v, dtype=self.dtype, device=self.device)
        return t.reshape((3,) + self.shape).contiguous()

    def close(self):
        if getattr(self, "handle", None) is not None:
            self.lib.cmlbm_mhd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def time(self):
        t = ctypes.c_int64()
        self._check(self.lib.cmlbm_mhd_get_time(self.handle, ctypes.byref(t)), "get_time")
        return t.value

    def init(self, b, u=None):
        bt, ut = self._vec(b), self._vec(u)
        self._check(self.lib.cmlbm_mhd_init(self.handle, _ptr(bt), _ptr(ut), self._stream()), "init")
        self.torch.cuda.current_stream(self.device).synchronize()

    def step(self, u=None):
        """One step with the fluid velocity u (device tensor, (3, nz, ny, nx) or
        a view of the fluid's (3, 1, nz, ny, nx) moments; None = rest)."""
        self._check(self.lib.cmlbm_mhd_step(self.handle, _ptr(self._vec(u)), self._stream()), "step")

    def fields(self, u=None, current="populations", F_out=None):
        """(b, j) as new tensors; with F_out (a contiguous device tensor of 3N
        values) the Lorentz force F = j x b is written there too."""
        b = self.torch.empty((3,) + self.shape, dtype=self.dtype, device=self.device)
        j = self.torch.empty_like(b)
        if F_out is not None:
            assert F_out.is_contiguous() and F_out.dtype == self.dtype and F_out.numel() == b.numel()
        self._check(self.lib.cmlbm_mhd_fields(self.handle, _ptr(self._vec(u)), CURRENT[current], _ptr(b), _ptr(j),
                                              _ptr(F_out), self._stream()), "fields")
        return b, j

    def populations(self):
        out = self.torch.empty((7, 3) + self.shape, dtype=self.torch.float64, device=self.device)
        self._check(self.lib.cmlbm_mhd_populations(self.handle, _ptr(out), self._stream()), "populations")
        return out

    def load_populations(self, h):
        t = self.torch.as_tensor(np.asarray(h) if isinstance(h, np.ndarray) else h, dtype=self.torch.float64,
                                 device=self.device).contiguous()
        self._check(self.lib.cmlbm_mhd_load_populations(self.handle, _ptr(t), self._stream()), "load_populations")
        self.torch.cuda.current_stream(self.device).synchronize()


class CoupledMHD:
    """The D3Q27 fluid (libcmlbm, one box) coupled to the magnetic lattice
    through the Lorentz force.  One step:
      (a) u_lag = fluid velocity with the force in effect (the previous step's);
      (b) b and j from the magnetic populations (j with u_lag); F = j x b
          written into the fluid's registered force field;
      (c) u = fluid velocity with F;
      (d) magnetic collision towards h^eq(b, u) and streaming;
      (e) fluid step with F.
    `model` is a fluid collision model of cmlbm.MODELS (m1, m4, m5, ...).
    `wall` flags axes with walls for both lattices (fluid: halfway
    bounce-back; field: b = b_wall there); `body_force` is a uniform force
    density added to the Lorentz force (the driving of a channel)."""

    def __init__(self, nx, ny, nz, tau, tau_m, storage="fp64", model="m1", current="populations", device="cuda:0",
                 wall=(0, 0, 0), b_wall=None, body_force=None):
        from .cmlbm import Lattice

        self.fluid = Lattice(nx, ny, nz, tau=tau, storage=storage, model=model, wall=wall, device=device)
        self.mag = MagneticLattice(nx, ny, nz, tau_m, storage=storage, device=device, wall=wall, b_wall=b_wall)
        if body_force is not None:
            self.mag.set_body_force(body_force)
        self.torch = self.mag.torch
        self.current = current
        self.shape = (int(nz), int(ny), int(nx))
        self.dtype = self.mag.dtype
        self.F = self.torch.zeros((3, 1) + self.shape, dtype=self.dtype, device=self.mag.device)

    def init(self, rho, u, b):
        u = np.asarray(u, np.float64).reshape((3,) + self.shape)
        self.fluid.init(np.asarray(rho, np.float64).reshape((1,) + self.shape), u.reshape((3, 1) + self.shape))
        self.F.zero_()
        self.fluid.set_force("field", field=self.F)
        self.F = self.fluid.force_field  # the buffer the fluid solver borrows
        self.mag.init(b, u)

    def velocity(self):
        dt = self.torch.float64 if self.dtype == self.torch.float64 else self.torch.float32
        return self.fluid.moments(dtype=dt)

    def step(self, n=1):
        for _ in range(int(n)):
            _, u_lag = self.velocity()
            self.mag.fields(u_lag, self.current, F_out=self.F)
            _, u = self.velocity()
            self.mag.step(u)
            self.fluid.step(1)

    @property
    def time(self):
        return self.fluid.time

    def state(self):
        """(rho, u, b, j) at the current time (j with the force in effect)."""
        rho, u = self.velocity()
        b, j = self.mag.fields(u, self.current)
        return rho.reshape(self.shape), u.reshape((3,) + self.shape), b, j
