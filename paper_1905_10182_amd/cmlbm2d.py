"""Python binding of libcmlbm2d (C ABI in include/cmlbm2d.h): the D2Q9
central-moment model with Hermite forcing of App. B.

Argument marshalling only: every step of the method runs in the HIP kernels
of libcmlbm2d.so.  PyTorch provides device memory and the current HIP stream.
If the library is missing this module raises; there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcmlbm2d.so")

OK, EINVAL, ENOMEM, EHIP, ESTATE = 0, -1, -2, -3, -5
FP64, FP32, FP16, BF16 = 0, 1, 2, 3
STORAGE = {"fp64": FP64, "fp32": FP32, "fp16": FP16, "bf16": BF16}
STORAGE_BYTES = {FP64: 8, FP32: 4, FP16: 2, BF16: 2}
FORCE_NONE, FORCE_UNIFORM, FORCE_FIELD = 0, 1, 2

# Every entry point declared in include/cmlbm2d.h.
EXPORTS = ["cmlbm2d_required_bytes", "cmlbm2d_create", "cmlbm2d_set_force", "cmlbm2d_init", "cmlbm2d_step",
           "cmlbm2d_moments", "cmlbm2d_populations", "cmlbm2d_load_populations", "cmlbm2d_get_time",
           "cmlbm2d_destroy", "cmlbm2d_last_error", "cmlbm2d_status_string"]


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("tau", ctypes.c_double),
                ("rho0", ctypes.c_double), ("storage", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class Cmlbm2dError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_status_string(code)}: {msg}")
        self.code = code


_lib = None


def load_library():
    """Load libcmlbm2d.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is missing: build it with `python -m paper_1905_10182_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32
    P = ctypes.POINTER(Params)
    lib.cmlbm2d_required_bytes.argtypes = [P, ctypes.POINTER(sz)]
    lib.cmlbm2d_create.argtypes = [P, vp, sz, vp, sz, ctypes.POINTER(vp)]
    lib.cmlbm2d_set_force.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), vp, ctypes.c_int, vp]
    lib.cmlbm2d_init.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    lib.cmlbm2d_step.argtypes = [vp, i32, vp]
    lib.cmlbm2d_moments.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    lib.cmlbm2d_populations.argtypes = [vp, vp, vp]
    lib.cmlbm2d_load_populations.argtypes = [vp, vp, vp]
    lib.cmlbm2d_get_time.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.cmlbm2d_destroy.argtypes = [vp]
    lib.cmlbm2d_last_error.argtypes = [vp]
    lib.cmlbm2d_last_error.restype = ctypes.c_char_p
    lib.cmlbm2d_status_string.argtypes = [ctypes.c_int]
    lib.cmlbm2d_status_string.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("cmlbm2d_last_error", "cmlbm2d_status_string"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _status_string(code):
    try:
        return load_library().cmlbm2d_status_string(code).decode()
    except OSError:
        return str(code)


def make_params(nx, ny, tau=0.8, rho0=1.0, storage="fp32", flags=0):
    p = Params()
    p.nx, p.ny = int(nx), int(ny)
    p.tau, p.rho0 = float(tau), float(rho0)
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.flags = int(flags)
    return p


def required_bytes(params):
    """Population buffer bytes; host-only."""
    n = ctypes.c_size_t()
    rc = load_library().cmlbm2d_required_bytes(ctypes.byref(params), ctypes.byref(n))
    if rc != OK:
        raise Cmlbm2dError(rc, "invalid lattice parameters")
    return n.value


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Lattice2D:
    """One D2Q9 handle over torch-allocated device buffers.

    Shapes on the Python side: scalar fields (ny, nx), vector fields
    (2, ny, nx), populations (9, ny, nx) in the velocity order of App. B.
    """

    def __init__(self, nx, ny, tau=0.8, rho0=1.0, storage="fp32", device="cuda"):
        import torch

        self.torch = torch
        self.lib = load_library()
        self.params = make_params(nx, ny, tau, rho0, storage)
        self.shape = (int(ny), int(nx))
        self.N = int(ny) * int(nx)
        self.storage = self.params.storage
        self.device = torch.device(device)
        self.pop_bytes = required_bytes(self.params)
        self._a = torch.empty(self.pop_bytes, dtype=torch.uint8, device=self.device)
        self._b = torch.empty(self.pop_bytes, dtype=torch.uint8, device=self.device)
        self._field = None
        h = ctypes.c_void_p()
        rc = self.lib.cmlbm2d_create(ctypes.byref(self.params), _ptr(self._a), self.pop_bytes, _ptr(self._b),
                                     self.pop_bytes, ctypes.byref(h))
        if rc != OK:
            raise Cmlbm2dError(rc, "cmlbm2d_create failed (alignment or size)")
        self.handle = h

    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _check(self, rc, what):
        if rc != OK:
            raise Cmlbm2dError(rc, f"{what}: {self.lib.cmlbm2d_last_error(self.handle).decode()}")

    def _dev(self, x, dtype, shape):
        if isinstance(x, np.ndarray) and not x.flags.writeable:
            x = np.array(x)  # torch refuses to wrap read-only (e.g. broadcast) arrays
        t = self.torch.as_tensor(x, dtype=dtype, device=self.device)
        t = t.expand(shape) if t.shape != shape else t
        return t.contiguous()

    def close(self):
        if getattr(self, "handle", None) is not None:
            self.lib.cmlbm2d_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def time(self):
        t = ctypes.c_int64()
        self._check(self.lib.cmlbm2d_get_time(self.handle, ctypes.byref(t)), "get_time")
        return t.value

    def set_force(self, mode, values=None, field=None):
        """mode: 'none' | 'uniform' (values[2]) | 'field' (field (2, ny, nx))."""
        m = {"none": FORCE_NONE, "uniform": FORCE_UNIFORM, "field": FORCE_FIELD}[mode]
        hv = None
        if values is not None:
            arr = np.ascontiguousarray(np.asarray(values, np.float64).ravel())
            hv = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        fptr, io = None, FP64
        if m == FORCE_FIELD:
            dt = self.torch.float64 if self.storage == FP64 else self.torch.float32
            io = FP64 if self.storage == FP64 else FP32
            self._field = self._dev(field, dt, (2,) + self.shape)
            fptr = _ptr(self._field)
        else:
            self._field = None
        self._check(self.lib.cmlbm2d_set_force(self.handle, m, hv, fptr, io, self._stream()), "set_force")

    def init(self, rho=None, u=None, dtype=None):
        dtype = dtype or self.torch.float64
        io = FP64 if dtype == self.torch.float64 else FP32
        r = None if rho is None else self._dev(rho, dtype, self.shape)
        v = None if u is None else self._dev(u, dtype, (2,) + self.shape)
        self._check(self.lib.cmlbm2d_init(self.handle, _ptr(r), _ptr(v), io, self._stream()), "init")
        self.torch.cuda.current_stream(self.device).synchronize()  # r, v alive until consumed

    def step(self, n=1):
        self._check(self.lib.cmlbm2d_step(self.handle, int(n), self._stream()), "step")

    def moments(self, dtype=None):
        dtype = dtype or self.torch.float64
        io = FP64 if dtype == self.torch.float64 else FP32
        rho = self.torch.empty(self.shape, dtype=dtype, device=self.device)
        u = self.torch.empty((2,) + self.shape, dtype=dtype, device=self.device)
        self._check(self.lib.cmlbm2d_moments(self.handle, _ptr(rho), _ptr(u), io, self._stream()), "moments")
        return rho, u

    def populations(self):
        out = self.torch.empty((9,) + self.shape, dtype=self.torch.float64, device=self.device)
        self._check(self.lib.cmlbm2d_populations(self.handle, _ptr(out), self._stream()), "populations")
        return out

    def load_populations(self, f):
        t = self._dev(f, self.torch.float64, (9,) + self.shape)
        self._check(self.lib.cmlbm2d_load_populations(self.handle, _ptr(t), self._stream()), "load_populations")
        self.torch.cuda.current_stream(self.device).synchronize()
