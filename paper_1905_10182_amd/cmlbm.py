"""Python binding of libcmlbm (C ABI in include/cmlbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
libcmlbm.so.  PyTorch provides device memory and the current HIP stream.  If
the library is missing this module raises; there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcmlbm.so")

OK, EINVAL, ENOMEM, EHIP, EUNSTABLE, ESTATE = 0, -1, -2, -3, -4, -5
FP64, FP32, FP16, BF16, MOM32 = 0, 1, 2, 3, 4
# population storage types, and the moment representation (nine FP32 numbers per cell)
STORAGE = {"fp64": FP64, "fp32": FP32, "fp16": FP16, "bf16": BF16, "mom32": MOM32}
STORAGE_BYTES = {FP64: 8, FP32: 4, FP16: 2, BF16: 2, MOM32: 4}
PERIODIC, BOUNCEBACK = 0, 1
FORCE_NONE, FORCE_UNIFORM, FORCE_BATCH, FORCE_PROFILE_Y, FORCE_FIELD = 0, 1, 2, 3, 4
FLAG_SOLID, FLAG_RESIDUAL, FLAG_STOCHASTIC, FLAG_FORCE_GUO, FLAG_EQ_SECOND, FLAG_BGK = 1, 2, 4, 8, 16, 32
FLAG_FUSED_REDUCE = 64
# collision models: the method (M1), the comparison models of Sec. III, and the
# single-relaxation-time controls (classical BGK with Guo forcing; BGK with the
# complete equilibrium and forcing)
MODELS = {"m1": 0, "m4": FLAG_FORCE_GUO, "m5": FLAG_FORCE_GUO | FLAG_EQ_SECOND, "eq2": FLAG_EQ_SECOND,
          "bgk": FLAG_BGK | FLAG_FORCE_GUO | FLAG_EQ_SECOND, "bgk6": FLAG_BGK}
REDUCE_RESIDUAL, REDUCE_SNAPSHOT = 1, 2
RED = {"mass": 0, "momx": 1, "momy": 2, "momz": 3, "ke": 4, "umax": 5, "nonfinite": 6, "fluid": 7,
       "du2": 8, "u2": 9, "residual": 10}
NRED = 11

# Every entry point declared in include/cmlbm.h.
EXPORTS = ["cmlbm_required_bytes", "cmlbm_create", "cmlbm_set_solid", "cmlbm_set_force", "cmlbm_init",
           "cmlbm_step", "cmlbm_moments", "cmlbm_reduce", "cmlbm_step_reduce", "cmlbm_populations",
           "cmlbm_load_populations",
           "cmlbm_save_state", "cmlbm_restore_state", "cmlbm_get_time", "cmlbm_set_time", "cmlbm_destroy",
           "cmlbm_last_error", "cmlbm_status_string", "cmlbm_pseudopotential_force", "cmlbm_device_copy", "cmlbm_plane_copy",
           "cmlbm_row_block_copy"]


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("nbatch", ctypes.c_int32), ("tau", ctypes.c_double), ("rho0", ctypes.c_double),
                ("storage", ctypes.c_int32), ("wall", ctypes.c_int32 * 3), ("flags", ctypes.c_uint32)]


class CmlbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_status_string(code)}: {msg}")
        self.code = code


_lib = None


def load_library():
    """Load libcmlbm.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is missing: build it with `python -m paper_1905_10182_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, u32, dp = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_uint32, ctypes.c_void_p
    P = ctypes.POINTER(Params)
    lib.cmlbm_required_bytes.argtypes = [P, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    lib.cmlbm_create.argtypes = [P, vp, sz, vp, sz, vp, sz, ctypes.POINTER(vp)]
    lib.cmlbm_set_solid.argtypes = [vp, vp, vp]
    lib.cmlbm_set_force.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), vp, ctypes.c_int, vp]
    lib.cmlbm_init.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    lib.cmlbm_step.argtypes = [vp, i32, vp]
    lib.cmlbm_moments.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    lib.cmlbm_reduce.argtypes = [vp, u32, ctypes.POINTER(ctypes.c_double), vp]
    lib.cmlbm_step_reduce.argtypes = [vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.cmlbm_pseudopotential_force.argtypes = [vp, ctypes.c_double, vp, ctypes.c_int, vp, vp]
    lib.cmlbm_populations.argtypes = [vp, dp, vp]
    lib.cmlbm_load_populations.argtypes = [vp, dp, vp]
    lib.cmlbm_save_state.argtypes = [vp, vp, sz, vp]
    lib.cmlbm_restore_state.argtypes = [vp, vp, sz, vp]
    lib.cmlbm_get_time.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.cmlbm_set_time.argtypes = [vp, ctypes.c_int64]
    lib.cmlbm_destroy.argtypes = [vp]
    lib.cmlbm_last_error.argtypes = [vp]
    lib.cmlbm_last_error.restype = ctypes.c_char_p
    lib.cmlbm_device_copy.argtypes = [vp, vp, sz, vp]
    lib.cmlbm_plane_copy.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, vp]
    lib.cmlbm_row_block_copy.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, vp]
    lib.cmlbm_status_string.argtypes = [ctypes.c_int]
    lib.cmlbm_status_string.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("cmlbm_last_error", "cmlbm_status_string"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _status_string(code):
    try:
        return load_library().cmlbm_status_string(code).decode()
    except OSError:
        return str(code)


def device_copy(dst, src, stream=None):
    """Copy tensor src into dst (same byte size, 16-byte aligned) with the
    library's 16-byte non-temporal copy kernel (a bandwidth measurement aid)."""
    import torch
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    s = torch.cuda.current_stream().cuda_stream if stream is None else stream
    rc = load_library().cmlbm_device_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                                          ctypes.c_void_p(s))
    if rc != OK:
        raise CmlbmError(rc, "device_copy")


def plane_copy(dst, src, planes, cells, plane_stride, stream=None):
    """dst[p * plane_stride + c] = src[p * plane_stride + c] for p < planes
    (9 or 27), c < cells, FP32 tensors on the GPU, with the library's plane
    copy kernel: the FP32 step's access pattern without its arithmetic (a
    bandwidth measurement aid)."""
    import torch
    span = (planes - 1) * plane_stride + cells
    assert src.dtype == torch.float32 and dst.dtype == torch.float32
    assert src.numel() >= span and dst.numel() >= span
    s = torch.cuda.current_stream().cuda_stream if stream is None else stream
    rc = load_library().cmlbm_plane_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), planes,
                                         cells, plane_stride, ctypes.c_void_p(s))
    if rc != OK:
        raise CmlbmError(rc, "plane_copy")


def row_block_copy(dst, src, rows, row_len, stream=None):
    """Copy rows * 27 * row_len FP32 values laid out as row blocks
    (population p of cell x in row r at (r * 27 + p) * row_len + x), one cell
    per lane, with the library's row-block copy kernel: the FP32 population
    step's access pattern without its arithmetic (a bandwidth measurement
    aid)."""
    import torch
    span = rows * 27 * row_len
    assert src.dtype == torch.float32 and dst.dtype == torch.float32
    assert src.numel() >= span and dst.numel() >= span
    s = torch.cuda.current_stream().cuda_stream if stream is None else stream
    rc = load_library().cmlbm_row_block_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), rows,
                                             row_len, ctypes.c_void_p(s))
    if rc != OK:
        raise CmlbmError(rc, "row_block_copy")


def make_params(nx, ny, nz, nbatch=1, tau=0.8, rho0=1.0, storage="fp32", wall=(0, 0, 0), flags=0):
    p = Params()
    p.nx, p.ny, p.nz, p.nbatch = int(nx), int(ny), int(nz), int(nbatch)
    p.tau, p.rho0 = float(tau), float(rho0)
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    for a in range(3):
        p.wall[a] = int(wall[a])
    p.flags = int(flags)
    return p


def required_bytes(params):
    """(population buffer bytes, scratch bytes); host-only."""
    lib = load_library()
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    rc = lib.cmlbm_required_bytes(ctypes.byref(params), ctypes.byref(a), ctypes.byref(b))
    if rc != OK:
        raise CmlbmError(rc, "invalid lattice parameters")
    return a.value, b.value


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Lattice:
    """One handle of the solver over torch-allocated device buffers.

    Shapes on the Python side: scalar fields (nbatch, nz, ny, nx), vector
    fields (3, nbatch, nz, ny, nx), populations (27, nbatch, nz, ny, nx).
    """

    def __init__(self, nx, ny, nz, nbatch=1, tau=0.8, rho0=1.0, storage="fp32", wall=(0, 0, 0),
                 solid=False, residual=False, stochastic=False, model="m1", fused_reduce=False, device="cuda"):
        import torch

        self.torch = torch
        self.lib = load_library()
        flags = (FLAG_SOLID if solid else 0) | (FLAG_RESIDUAL if residual else 0) | \
            (FLAG_STOCHASTIC if stochastic else 0) | MODELS[model] | (FLAG_FUSED_REDUCE if fused_reduce else 0)
        self.params = make_params(nx, ny, nz, nbatch, tau, rho0, storage, wall, flags)
        self.shape = (int(nbatch), int(nz), int(ny), int(nx))
        self.N = int(np.prod(self.shape))
        self.storage = self.params.storage
        self.device = torch.device(device)
        pop_bytes, scratch_bytes = required_bytes(self.params)
        self.pop_bytes, self.scratch_bytes = pop_bytes, scratch_bytes
        self._a = torch.empty(pop_bytes, dtype=torch.uint8, device=self.device)
        self._b = torch.empty(pop_bytes, dtype=torch.uint8, device=self.device)
        self._s = torch.empty(max(scratch_bytes, 256), dtype=torch.uint8, device=self.device)
        self._field = None
        h = ctypes.c_void_p()
        rc = self.lib.cmlbm_create(ctypes.byref(self.params), _ptr(self._a), pop_bytes, _ptr(self._b), pop_bytes,
                                   _ptr(self._s), self._s.numel(), ctypes.byref(h))
        if rc != OK:
            raise CmlbmError(rc, "cmlbm_create failed (alignment or size)")
        self.handle = h

    # -- plumbing
    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _check(self, rc, what):
        if rc != OK:
            msg = self.lib.cmlbm_last_error(self.handle).decode()
            raise CmlbmError(rc, f"{what}: {msg}")

    def _dev(self, x, dtype, shape):
        t = self.torch.as_tensor(x, dtype=dtype, device=self.device)
        t = t.expand(shape) if t.shape != shape else t
        return t.contiguous()

    def close(self):
        if getattr(self, "handle", None) is not None:
            self.lib.cmlbm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- API
    @property
    def time(self):
        t = ctypes.c_int64()
        self._check(self.lib.cmlbm_get_time(self.handle, ctypes.byref(t)), "get_time")
        return t.value

    @time.setter
    def time(self, t):
        self._check(self.lib.cmlbm_set_time(self.handle, int(t)), "set_time")

    def set_solid(self, solid):
        """solid: (nbatch, nz, ny, nx) bool/uint8 array, or None to clear."""
        t = None if solid is None else self._dev(solid, self.torch.uint8, self.shape)
        self._check(self.lib.cmlbm_set_solid(self.handle, _ptr(t), self._stream()), "set_solid")

    @property
    def force_field(self):
        """The device tensor the solver borrows in FIELD mode (writing into it
        changes the force of later steps and moments), else None."""
        return self._field

    def set_force(self, mode, values=None, field=None):
        """mode: 'none' | 'uniform' (values[3]) | 'batch' (values[nbatch][3]) |
        'profile_y' (values[ny][3]) | 'field' (field (3, nbatch, nz, ny, nx))."""
        m = {"none": FORCE_NONE, "uniform": FORCE_UNIFORM, "batch": FORCE_BATCH, "profile_y": FORCE_PROFILE_Y,
             "field": FORCE_FIELD}[mode]
        hv = None
        if values is not None:
            arr = np.ascontiguousarray(np.asarray(values, np.float64).ravel())
            self._force_host = arr
            hv = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        fptr, io = None, FP64
        if m == FORCE_FIELD:
            dt = self.torch.float64 if self.storage == FP64 else self.torch.float32
            io = FP64 if self.storage == FP64 else FP32
            self._field = self._dev(field, dt, (3,) + self.shape)
            fptr = _ptr(self._field)
        else:
            self._field = None
        self._check(self.lib.cmlbm_set_force(self.handle, m, hv, fptr, io, self._stream()), "set_force")

    def init(self, rho=None, u=None, dtype=None):
        dtype = dtype or self.torch.float64
        io = FP64 if dtype == self.torch.float64 else FP32
        r = None if rho is None else self._dev(rho, dtype, self.shape)
        v = None if u is None else self._dev(u, dtype, (3,) + self.shape)
        self._check(self.lib.cmlbm_init(self.handle, _ptr(r), _ptr(v), io, self._stream()), "init")
        self._keep = (r, v)  # alive until the stream has consumed them
        self.torch.cuda.current_stream(self.device).synchronize()
        self._keep = None

    def step(self, n=1):
        self._check(self.lib.cmlbm_step(self.handle, int(n), self._stream()), "step")

    def moments(self, dtype=None):
        dtype = dtype or self.torch.float64
        io = FP64 if dtype == self.torch.float64 else FP32
        rho = self.torch.empty(self.shape, dtype=dtype, device=self.device)
        u = self.torch.empty((3,) + self.shape, dtype=dtype, device=self.device)
        self._check(self.lib.cmlbm_moments(self.handle, _ptr(rho), _ptr(u), io, self._stream()), "moments")
        return rho, u

    def density(self, dtype=None, out=None):
        """rho(x, t) alone: the moment export without the velocity (into out if given)."""
        dtype = dtype or self.torch.float64
        io = FP64 if dtype == self.torch.float64 else FP32
        if out is None:
            out = self.torch.empty(self.shape, dtype=dtype, device=self.device)
        assert out.dtype == dtype and out.is_contiguous() and tuple(out.shape) == self.shape
        self._check(self.lib.cmlbm_moments(self.handle, _ptr(out), None, io, self._stream()), "moments")
        return out

    def populations(self):
        out = self.torch.empty((27,) + self.shape, dtype=self.torch.float64, device=self.device)
        self._check(self.lib.cmlbm_populations(self.handle, _ptr(out), self._stream()), "populations")
        return out

    def load_populations(self, f):
        t = self._dev(f, self.torch.float64, (27,) + self.shape)
        self._check(self.lib.cmlbm_load_populations(self.handle, _ptr(t), self._stream()), "load_populations")
        self.torch.cuda.current_stream(self.device).synchronize()

    def save_state(self):
        """Bitwise checkpoint: (opaque device blob, step counter)."""
        blob = self.torch.empty(self.pop_bytes, dtype=self.torch.uint8, device=self.device)
        self._check(self.lib.cmlbm_save_state(self.handle, _ptr(blob), blob.numel(), self._stream()), "save_state")
        return blob, self.time

    def restore_state(self, blob, t=None):
        self._check(self.lib.cmlbm_restore_state(self.handle, _ptr(blob), blob.numel(), self._stream()),
                    "restore_state")
        if t is not None:
            self.time = t

    def pseudopotential_force(self, G, rho, out=None):
        """Shan-Chen force -G psi sum_i w_i c_i psi(x + c_i), psi = 1 - exp(-rho), from a
        device density field (as returned by moments(); FP64 for FP64 storage, FP32
        otherwise); returns (or fills) the force field (3, nbatch, nz, ny, nx)."""
        dt = self.torch.float64 if self.storage == FP64 else self.torch.float32
        io = FP64 if self.storage == FP64 else FP32
        r = self._dev(rho, dt, self.shape)
        if out is None:
            out = self.torch.empty((3,) + self.shape, dtype=dt, device=self.device)
        assert out.dtype == dt and out.is_contiguous() and tuple(out.shape) == (3,) + self.shape
        self._check(self.lib.cmlbm_pseudopotential_force(self.handle, float(G), _ptr(r), io, _ptr(out),
                                                         self._stream()), "pseudopotential_force")
        return out

    def step_reduce(self, allow_unstable=False):
        """One step that also returns the FP64 reductions of the state it
        started from (numpy (nbatch, NRED), as reduce()); needs
        fused_reduce=True."""
        out = np.zeros((self.shape[0], NRED), np.float64)
        rc = self.lib.cmlbm_step_reduce(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        self._stream())
        if rc == EUNSTABLE and allow_unstable:
            return out
        self._check(rc, "step_reduce")
        return out

    def reduce(self, residual=False, snapshot=False, allow_unstable=False):
        """FP64 reductions, numpy array (nbatch, NRED) laid out as RED."""
        out = np.zeros((self.shape[0], NRED), np.float64)
        what = (REDUCE_RESIDUAL if residual else 0) | (REDUCE_SNAPSHOT if snapshot else 0)
        rc = self.lib.cmlbm_reduce(self.handle, what, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   self._stream())
        if rc == EUNSTABLE and allow_unstable:
            return out
        self._check(rc, "reduce")
        return out
