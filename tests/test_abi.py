"""CPU-side checks of the C ABI (include/cmlbm.h): the library loads, exports
every declared entry point, and rejects invalid arguments on the host before
any device work.  No call here reaches the GPU."""
import ctypes
import os
import re

import pytest

from paper_1905_10182_amd import cmlbm as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cmlbm.h")


@pytest.fixture(scope="module")
def lib():
    return B.load_library()


def declared_functions(path):
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cmlbm_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions(HEADER) == sorted(B.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions(HEADER):
        assert hasattr(lib, name), name


def test_status_strings(lib):
    assert lib.cmlbm_status_string(0) == b"CMLBM_OK"
    assert lib.cmlbm_status_string(-4) == b"CMLBM_EUNSTABLE"
    assert lib.cmlbm_status_string(17) == b"CMLBM_UNKNOWN"
    assert lib.cmlbm_last_error(None) == b""


def req(**kw):
    base = dict(nx=32, ny=16, nz=16, nbatch=1, tau=0.8, rho0=1.0, storage="fp32", wall=(0, 0, 0), flags=0)
    base.update(kw)
    return B.make_params(**base)


PLANE_PAD = 4096  # bytes between consecutive moment planes


def test_required_bytes_padding():
    # rows padded to 256 bytes; population storage: one block of 27 population rows per lattice row
    pop, scratch = B.required_bytes(req(nx=32, storage="fp32"))
    assert pop == 16 * 16 * 27 * 64 * 4
    pop, _ = B.required_bytes(req(nx=256, ny=256, nz=256, storage="fp32"))
    assert pop == 27 * 256 ** 3 * 4
    pop, _ = B.required_bytes(req(nx=512, ny=512, nz=512, storage="fp16"))
    assert pop == 27 * 512 ** 3 * 2
    pop, _ = B.required_bytes(req(nx=37, ny=13, nz=11, nbatch=2, storage="fp64"))
    assert pop == 13 * 11 * 2 * 27 * 64 * 8
    pop, _ = B.required_bytes(req(nx=3, ny=5, nz=7, storage="bf16"))
    assert pop == -(-(5 * 7 * 27 * 128 * 2) // 256) * 256
    # a mask (walls/solid) and the residual snapshot enlarge the scratch
    _, s0 = B.required_bytes(req())
    _, s1 = B.required_bytes(req(wall=(0, 1, 0)))
    _, s2 = B.required_bytes(req(flags=B.FLAG_RESIDUAL))
    assert s1 >= s0 + 16 * 16 * 64 * 4
    assert s2 >= s0 + 3 * 32 * 16 * 16 * 8


def test_plane_size_limit():
    # one population's values (and the link mask) are indexed with 32-bit byte offsets: 1024^3 FP32
    # (4 GiB per population) is refused, FP16 accepted
    with pytest.raises(B.CmlbmError):
        B.required_bytes(req(nx=1024, ny=1024, nz=1024, storage="fp32"))
    pop, _ = B.required_bytes(req(nx=1024, ny=1024, nz=1024, storage="fp16"))
    assert pop == 27 * 1024 ** 3 * 2


@pytest.mark.parametrize("kw", [dict(tau=0.5), dict(tau=0.3), dict(tau=float("nan")), dict(nx=0), dict(ny=-1),
                                dict(nbatch=0), dict(rho0=0.0), dict(storage=7), dict(wall=(2, 0, 0)),
                                dict(flags=8, storage="fp16"), dict(flags=16, storage="bf16"),
                                dict(nz=1, wall=(0, 0, 1)), dict(storage="mom32", wall=(0, 1, 0)),
                                dict(storage="mom32", flags=1), dict(storage="mom32", flags=4),
                                dict(storage="mom32", flags=8), dict(storage=5), dict(flags=32 | 8),
                                dict(flags=32, storage="fp16"), dict(flags=128)])
def test_invalid_params(kw):
    with pytest.raises(B.CmlbmError) as e:
        B.required_bytes(req(**kw))
    assert e.value.code == B.EINVAL


def create(lib, params, a, na, b, nb, s, ns):
    h = ctypes.c_void_p()
    rc = lib.cmlbm_create(ctypes.byref(params), a, na, b, nb, s, ns, ctypes.byref(h))
    return rc, h


def test_create_validates_buffers(lib):
    p = req()
    pop, scr = B.required_bytes(p)
    A, Bp, S = 0x10000000, 0x20000000, 0x30000000  # never dereferenced: create is host-only
    assert create(lib, p, None, pop, Bp, pop, S, scr)[0] == B.EINVAL
    assert create(lib, p, A, pop, A, pop, S, scr)[0] == B.EINVAL
    assert create(lib, p, A + 8, pop, Bp, pop, S, scr)[0] == B.EINVAL
    assert create(lib, p, A, pop - 1, Bp, pop, S, scr)[0] == B.ENOMEM
    assert create(lib, p, A, pop, Bp, pop, S, scr - 1)[0] == B.ENOMEM
    rc, h = create(lib, p, A, pop, Bp, pop, S, scr)
    assert rc == B.OK and h.value
    # state checks happen before any device call
    assert lib.cmlbm_step(h, 1, None) == B.ESTATE
    assert b"before init" in lib.cmlbm_last_error(h)
    assert lib.cmlbm_step(h, -1, None) == B.EINVAL
    assert lib.cmlbm_moments(h, None, None, 5, None) == B.EINVAL
    out = (ctypes.c_double * B.NRED)()
    assert lib.cmlbm_reduce(h, 0, out, None) == B.ESTATE
    assert lib.cmlbm_reduce(h, 8, out, None) == B.EINVAL
    assert lib.cmlbm_set_solid(h, None, None) == B.ESTATE  # no CMLBM_FLAG_SOLID
    assert lib.cmlbm_set_force(h, 99, None, None, 0, None) == B.EINVAL
    assert lib.cmlbm_set_force(h, B.FORCE_UNIFORM, None, None, 0, None) == B.EINVAL
    assert lib.cmlbm_set_force(h, B.FORCE_FIELD, None, None, B.FP32, None) == B.EINVAL
    assert lib.cmlbm_set_force(h, B.FORCE_FIELD, None, ctypes.c_void_p(0x40000000), B.FP64, None) == B.EINVAL
    t = ctypes.c_int64()
    assert lib.cmlbm_get_time(h, ctypes.byref(t)) == B.OK and t.value == 0
    assert lib.cmlbm_set_time(h, 12) == B.OK
    assert lib.cmlbm_get_time(h, ctypes.byref(t)) == B.OK and t.value == 12
    assert lib.cmlbm_set_time(h, -1) == B.EINVAL
    assert lib.cmlbm_destroy(h) == B.OK
    assert lib.cmlbm_destroy(None) == B.OK


def test_null_handle_is_einval(lib):
    assert lib.cmlbm_step(None, 1, None) == B.EINVAL
    assert lib.cmlbm_init(None, None, None, 0, None) == B.EINVAL
    assert lib.cmlbm_populations(None, None, None) == B.EINVAL


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(OSError):
        B.load_library()


def test_moment_storage_bytes():
    """The moment representation keeps nine FP32 planes per buffer."""
    pop, _ = B.required_bytes(req(nx=64, ny=8, nz=8, storage="mom32"))
    assert pop == 9 * (8 * 8 * 64 * 4 + PLANE_PAD)
    pop32, _ = B.required_bytes(req(nx=64, ny=8, nz=8, storage="fp32"))
    assert pop32 == 27 * 8 * 8 * 64 * 4
    B.required_bytes(req(storage="mom32", flags=B.FLAG_RESIDUAL))  # residual snapshots are allowed


def test_fused_reduce_flag():
    # the per-wave partials: 10 doubles per 64-cell (16-bit: 128-cell) row segment
    _, base = B.required_bytes(req(nx=100, ny=8, nz=4, storage="fp32"))
    _, fused = B.required_bytes(req(nx=100, ny=8, nz=4, storage="fp32", flags=B.FLAG_FUSED_REDUCE))
    assert fused - base >= 2 * 8 * 4 * 10 * 8
    _, f16 = B.required_bytes(req(nx=256, ny=8, nz=4, storage="fp16", flags=B.FLAG_FUSED_REDUCE))
    _, b16 = B.required_bytes(req(nx=256, ny=8, nz=4, storage="fp16"))
    assert f16 - b16 >= 2 * 8 * 4 * 10 * 8
    # only with the method's collision on population storage
    for kw in (dict(storage="mom32"), dict(flags=B.FLAG_FUSED_REDUCE | B.FLAG_FORCE_GUO)):
        p = req(**kw)
        p.flags |= B.FLAG_FUSED_REDUCE
        with pytest.raises(B.CmlbmError):
            B.required_bytes(p)


def test_device_copy_validation(lib):
    base = 1 << 24  # stand-in device addresses: every call below fails validation before any launch
    P = lambda off: ctypes.c_void_p(base + off)
    assert lib.cmlbm_device_copy(None, P(0), 16, None) == B.EINVAL
    assert lib.cmlbm_device_copy(P(4096), None, 16, None) == B.EINVAL
    assert lib.cmlbm_device_copy(P(4096), P(8), 16, None) == B.EINVAL     # misaligned source
    assert lib.cmlbm_device_copy(P(4096 + 4), P(0), 16, None) == B.EINVAL  # misaligned destination
    assert lib.cmlbm_device_copy(P(4096), P(0), 24, None) == B.EINVAL     # not a multiple of 16 bytes
    assert lib.cmlbm_device_copy(P(4096), P(0), 0, None) == B.EINVAL
    assert lib.cmlbm_device_copy(P(64), P(0), 128, None) == B.EINVAL      # overlapping


def test_plane_copy_validation(lib):
    """Argument checks of the plane copy, all before any GPU call."""
    P = ctypes.c_void_p
    lib.cmlbm_plane_copy.argtypes = [P, P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, P]
    far = 1 << 40
    assert lib.cmlbm_plane_copy(None, P(0x1000), 27, 64, 64, None) == B.EINVAL
    assert lib.cmlbm_plane_copy(P(far), None, 27, 64, 64, None) == B.EINVAL
    assert lib.cmlbm_plane_copy(P(far), P(0x1000), 8, 64, 64, None) == B.EINVAL     # planes: 9 or 27
    assert lib.cmlbm_plane_copy(P(far), P(0x1000), 27, 0, 64, None) == B.EINVAL     # no cells
    assert lib.cmlbm_plane_copy(P(far), P(0x1000), 27, 64, 63, None) == B.EINVAL    # stride below the cells
    assert lib.cmlbm_plane_copy(P(far + 2), P(0x1000), 27, 64, 64, None) == B.EINVAL  # misaligned
    assert lib.cmlbm_plane_copy(P(0x1000 + 256), P(0x1000), 9, 64, 64, None) == B.EINVAL  # overlapping


def test_row_block_copy_validation(lib):
    """Argument checks of the row-block copy, all before any GPU call."""
    P = ctypes.c_void_p
    lib.cmlbm_row_block_copy.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32, P]
    far = 1 << 44
    assert lib.cmlbm_row_block_copy(None, P(0x1000), 4, 64, None) == B.EINVAL
    assert lib.cmlbm_row_block_copy(P(far), None, 4, 64, None) == B.EINVAL
    assert lib.cmlbm_row_block_copy(P(far), P(0x1000), 0, 64, None) == B.EINVAL      # no rows
    assert lib.cmlbm_row_block_copy(P(far), P(0x1000), 4, 0, None) == B.EINVAL       # empty rows
    assert lib.cmlbm_row_block_copy(P(far + 2), P(0x1000), 4, 64, None) == B.EINVAL  # misaligned
    assert lib.cmlbm_row_block_copy(P(0x1000 + 27 * 64 * 4 * 4 - 4), P(0x1000), 4, 64, None) == B.EINVAL  # overlap
    assert lib.cmlbm_row_block_copy(P(far), P(0x1000), (1 << 40) // (27 * 4 * 64), 64, None) == B.EINVAL  # 2^40 B
