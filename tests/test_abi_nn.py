"""CPU-side checks of the C ABI of the warm-start network kernels
(include/cmnn.h): the library loads, exports every declared entry point, and
rejects invalid arguments on the host before any device work.  Every call
here is invalid, so none reaches a kernel launch."""
import ctypes
import os
import re

import pytest

from paper_1905_10182_amd import cmnn as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cmnn.h")
EINVAL = -1

P = ctypes.c_void_p(1 << 20)        # stand-in device pointers: never dereferenced (validation fails first)
P2 = ctypes.c_void_p((1 << 20) + 256)
ODD = ctypes.c_void_p((1 << 20) + 8)  # not 16-byte aligned
NULL = None


@pytest.fixture(scope="module")
def lib():
    return N.load_library()


def declared_functions(path):
    text = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
    return sorted(set(re.findall(r"\b(cmnn_[a-z0-9_]+)\s*\(", text)))


def g(n=2, d=8, h=8, w=16, periodic=(1, 0, 1)):
    return ctypes.byref(N.geom(n, d, h, w, periodic))


def test_header_and_binding_agree():
    assert declared_functions(HEADER) == sorted(N.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions(HEADER):
        assert hasattr(lib, name), name


def test_conv_forward_and_data_gradient_validation(lib):
    ok = dict(x=P, cin=32, w=P2, b=NULL, cout=32, act=1, y=P)
    def fwd(geom=None, **kw):
        a = dict(ok, **kw)
        return lib.cmnn_conv3d_fwd(geom if geom is not None else g(n=0), a["x"], a["cin"], a["w"], a["b"], a["cout"],
                                   a["act"], a["y"], NULL)
    assert fwd() == EINVAL  # empty batch
    for kw in (dict(cin=48), dict(cout=0), dict(cin=-32), dict(x=NULL), dict(w=NULL), dict(y=NULL), dict(x=ODD),
               dict(w=ODD), dict(act=2), dict(act=-1)):
        assert fwd(g(), **kw) == EINVAL, kw
    for geom in (g(d=0), g(h=-1), g(n=1024, d=1024, h=1024, w=2)):  # the last has 2^31 voxels
        assert fwd(geom) == EINVAL
    assert lib.cmnn_conv3d_fwd(None, P, 32, P2, NULL, 32, 1, P, NULL) == EINVAL
    assert lib.cmnn_conv3d_bwd_data(g(), P, 32, P2, 40, P, NULL) == EINVAL
    assert lib.cmnn_conv3d_bwd_data(g(), ODD, 32, P2, 32, P, NULL) == EINVAL
    assert lib.cmnn_conv3d_bwd_data(g(), P, 32, NULL, 32, P, NULL) == EINVAL
    assert lib.cmnn_conv3d_bwd_data(g(w=0), P, 32, P2, 32, P, NULL) == EINVAL

    # the data gradient with the activation gradient fused in
    L = lib.cmnn_conv3d_bwd_data_act
    assert L(g(), P, 32, P2, 40, P2, 1, P, NULL) == EINVAL        # channels not a multiple of 32
    assert L(g(), ODD, 32, P2, 32, P2, 1, P, NULL) == EINVAL      # misaligned dy
    assert L(g(), P, 32, P2, 32, NULL, 1, P, NULL) == EINVAL      # leaky needs its gate
    assert L(g(), P, 32, P2, 32, ODD, 1, P, NULL) == EINVAL       # misaligned gate
    assert L(g(), P, 32, P2, 32, P, 1, P, NULL) == EINVAL         # gate aliasing dx
    assert L(g(), P, 32, P2, 32, P2, 2, P, NULL) == EINVAL        # unknown activation
    assert L(g(w=0), P, 32, P2, 32, P2, 1, P, NULL) == EINVAL


def test_weight_gradient_workspace_and_validation(lib):
    n = ctypes.c_size_t()
    # brick geometry 16 x 32 x 32 x 64, 32 x 32 channels: 4096 bricks in 256
    # chunks, 27 x 32 x 32 FP32 partials each, plus the bias column partials
    assert lib.cmnn_conv3d_bwd_weight_workspace(ctypes.byref(N.geom(16, 32, 32, 64)), 32, 32, ctypes.byref(n)) == 0
    assert n.value == 256 * 27 * 32 * 32 * 4 + 1024 * 32 * 4
    # four 32 x 32 channel tiles: 64 chunks
    assert lib.cmnn_conv3d_bwd_weight_workspace(ctypes.byref(N.geom(16, 32, 32, 64)), 64, 64, ctypes.byref(n)) == 0
    assert n.value == 64 * 27 * 64 * 64 * 4 + 1024 * 64 * 4
    assert lib.cmnn_conv3d_bwd_weight_workspace(g(), 33, 32, ctypes.byref(n)) == EINVAL
    assert lib.cmnn_conv3d_bwd_weight_workspace(g(), 32, 32, None) == EINVAL
    assert lib.cmnn_conv3d_bwd_weight_workspace(g(n=0), 32, 32, ctypes.byref(n)) == EINVAL
    assert lib.cmnn_conv3d_bwd_weight_workspace(g(), 32, 32, ctypes.byref(n)) == 0
    need = n.value
    call = lambda **kw: lib.cmnn_conv3d_bwd_weight(g(), kw.get("x", P), 32, kw.get("dy", P2), kw.get("cout", 32),
                                                   kw.get("dw", P), NULL, kw.get("ws", P), kw.get("wsb", need), NULL)
    for kw in (dict(wsb=need - 1), dict(ws=NULL), dict(x=NULL), dict(dy=NULL), dict(dw=NULL), dict(x=ODD),
               dict(dy=ODD), dict(cout=288)):
        assert call(**kw) == EINVAL, kw


def test_weight_gradient_noalloc_validation(lib):
    """The no-allocation weight gradient refuses, before any device call, a
    geometry whose workspace exceeds its fixed 64 MiB scratch and invalid
    pointers or channel counts."""
    n = ctypes.c_size_t()
    big = N.geom(4, 3, 5, 4400, periodic=(1, 1, 1))  # generic kernel, 64 chunks of 27 x 160 x 160 partials
    assert lib.cmnn_conv3d_bwd_weight_workspace(ctypes.byref(big), 160, 160, ctypes.byref(n)) == 0
    assert n.value > 64 << 20
    assert lib.cmnn_conv3d_bwd_weight_noalloc(ctypes.byref(big), P, 160, P2, 160, P, NULL, NULL) == EINVAL
    call = lambda **kw: lib.cmnn_conv3d_bwd_weight_noalloc(g(), kw.get("x", P), 32, kw.get("dy", P2),
                                                           kw.get("cout", 32), kw.get("dw", P), NULL, NULL)
    for kw in (dict(x=NULL), dict(dy=NULL), dict(dw=NULL), dict(x=ODD), dict(dy=ODD), dict(cout=288),
               dict(cout=33)):
        assert call(**kw) == EINVAL, kw


def test_elementwise_validation(lib):
    assert lib.cmnn_act_bwd(P, P, NULL, 64, 1, NULL) == EINVAL
    assert lib.cmnn_act_bwd(P, P, P, 64, 3, NULL) == EINVAL
    assert lib.cmnn_pool2_fwd(g(d=7), P, 32, P2, NULL) == EINVAL  # odd extent
    assert lib.cmnn_pool2_fwd(g(), P, 0, P2, NULL) == EINVAL
    assert lib.cmnn_pool2_bwd(g(w=15), P, 32, P2, NULL) == EINVAL
    assert lib.cmnn_up2_fwd(g(), NULL, 32, P2, NULL) == EINVAL
    assert lib.cmnn_up2_bwd(g(h=0), P, 32, P2, NULL) == EINVAL
    assert lib.cmnn_concat_fwd(10, P, 0, P, 32, P2, NULL) == EINVAL
    assert lib.cmnn_concat_fwd(10, P, 32, NULL, 32, P2, NULL) == EINVAL
    assert lib.cmnn_concat_bwd(10, NULL, 32, 32, P, P2, NULL) == EINVAL
    assert lib.cmnn_concat_bwd(10, P, 32, -8, P, P2, NULL) == EINVAL
    assert lib.cmnn_add(10, P, NULL, P2, NULL) == EINVAL
    assert lib.cmnn_pack_weights(P, 0, 32, P, P2, NULL) == EINVAL
    assert lib.cmnn_pack_weights(P, 32, 32, P, NULL, NULL) == EINVAL
    assert lib.cmnn_pack_channels(10, P, 4, P2, 3, NULL) == EINVAL  # fewer slots than channels
    assert lib.cmnn_unpack_channels(10, P, 32, NULL, 4, NULL) == EINVAL
    assert lib.cmnn_adam(10, P, P, P, P, ctypes.c_float(1e-3), ctypes.c_float(0.9), ctypes.c_float(0.999),
                         ctypes.c_float(1e-8), ctypes.c_float(0.0), 0, NULL) == EINVAL  # step counts from 1


def test_skip_join_validation(lib):
    U, B, J = lib.cmnn_up2_concat_fwd, lib.cmnn_up2_bwd_act, lib.cmnn_pool2_bwd_add_act
    assert U(g(), P, 40, P2, 64, P, NULL) == EINVAL           # channels not a multiple of 32
    assert U(g(), P, 32, P2, 0, P, NULL) == EINVAL
    assert U(g(), ODD, 32, P2, 64, P, NULL) == EINVAL         # misaligned skip
    assert U(g(), P, 32, NULL, 64, P, NULL) == EINVAL
    assert U(g(n=1 << 12, d=64, h=64, w=32), P, 32, P2, 64, P, NULL) == EINVAL  # fine level over 2^31 - 1 voxels
    assert B(g(), P, 32, 64, P2, 1, P, NULL) == EINVAL        # stride below the channel count
    assert B(g(), P, 100, 64, P2, 1, P, NULL) == EINVAL       # stride not a multiple of 8
    assert B(g(), ODD, 96, 64, P2, 1, P, NULL) == EINVAL      # misaligned part pointer
    assert B(g(), P, 96, 64, NULL, 1, P, NULL) == EINVAL      # leaky needs its gate
    assert B(g(), P, 96, 64, ODD, 1, P, NULL) == EINVAL       # misaligned gate
    assert B(g(), P, 96, 64, P2, 2, P, NULL) == EINVAL        # unknown activation
    assert B(g(), P, 96, 64, P2, 1, NULL, NULL) == EINVAL
    assert J(g(d=7), P, 32, P2, 96, P2, 1, P, NULL) == EINVAL  # odd extent
    assert J(g(), P, 48, P2, 96, P2, 1, P, NULL) == EINVAL
    assert J(g(), P, 32, P2, 16, P2, 1, P, NULL) == EINVAL    # skip stride below the channel count
    assert J(g(), P, 32, ODD, 96, P2, 1, P, NULL) == EINVAL   # misaligned skip
    assert J(g(), P, 32, P2, 96, NULL, 1, P, NULL) == EINVAL
    assert J(g(), P, 32, P2, 96, P2, -1, P, NULL) == EINVAL
    assert J(g(), NULL, 32, P2, 96, P2, 1, P, NULL) == EINVAL


def test_bottleneck_join_validation(lib):
    n = ctypes.c_size_t()
    assert lib.cmnn_channel_mean_workspace(g(), 96, ctypes.byref(n)) == 0
    W = n.value
    MC, MA = lib.cmnn_channel_mean_concat, lib.cmnn_channel_mean_add_act
    assert MC(g(), P, 40, P2, P, W, NULL) == EINVAL            # channels not a multiple of 32
    assert MC(g(), P, 288, P2, P, 1 << 30, NULL) == EINVAL     # more than 256 channels
    assert MC(g(), ODD, 96, P2, P, W, NULL) == EINVAL
    assert MC(g(), P, 96, P2, P, W - 4, NULL) == EINVAL        # workspace too small
    assert MC(g(), P, 96, P2, NULL, W, NULL) == EINVAL
    assert MA(g(), P, 64, 96, P2, 192, P, 1, P2, P, W, NULL) == EINVAL    # dy stride below the channels
    assert MA(g(), P, 192, 96, P2, 100, P, 1, P2, P, W, NULL) == EINVAL   # skip stride not a multiple of 8
    assert MA(g(), P, 192, 96, NULL, 192, P, 1, P2, P, W, NULL) == EINVAL  # the skip part is required
    assert MA(g(), P, 192, 96, P2, 192, NULL, 1, P2, P, W, NULL) == EINVAL  # leaky needs its gate
    assert MA(g(), P, 192, 96, P2, 192, P, 1, ODD, P, W, NULL) == EINVAL
    assert MA(g(), P, 192, 96, P2, 192, P, 1, P2, P, W - 4, NULL) == EINVAL


def test_gather_validation(lib):
    GS, GP = lib.cmnn_gather_samples, lib.cmnn_gather_pack_channels
    assert GS(0, P, 64, P2, 4, 3, P, NULL) == EINVAL      # empty selection
    assert GS(2, NULL, 64, P2, 4, 3, P, NULL) == EINVAL   # no index array
    assert GS(2, P, 0, P2, 4, 3, P, NULL) == EINVAL
    assert GS(2, P, 64, P2, 0, 3, P, NULL) == EINVAL      # empty source
    assert GS(2, P, 64, P2, 4, 0, P, NULL) == EINVAL
    assert GS(2, P, 64, NULL, 4, 3, P, NULL) == EINVAL
    assert GP(2, P, 64, P2, 4, 2, P, 12, NULL) == EINVAL  # packed width not a multiple of 8
    assert GP(2, P, 64, P2, 4, 40, P, 32, NULL) == EINVAL  # fewer slots than channels
    assert GP(2, P, 64, P2, 4, 2, ODD, 32, NULL) == EINVAL
    assert GP(-1, P, 64, P2, 4, 2, P, 32, NULL) == EINVAL


def test_pack_batch_validation(lib):
    jobs = (N.PackJob * (N.PACK_MAX + 1))()
    for j in jobs:
        j.w, j.w_fwd, j.w_t, j.cin, j.cout = 1 << 20, (1 << 20) + 4096, (1 << 20) + 8192, 32, 32
    B = lib.cmnn_pack_weights_batch
    assert B(0, jobs, NULL) == EINVAL
    assert B(N.PACK_MAX + 1, jobs, NULL) == EINVAL  # more layers than one launch takes
    assert B(2, None, NULL) == EINVAL
    jobs[1].w_t = None
    assert B(2, jobs, NULL) == EINVAL
    jobs[1].w_t, jobs[0].cout = (1 << 20) + 8192, 0
    assert B(2, jobs, NULL) == EINVAL


def test_reduction_workspaces_and_validation(lib):
    n = ctypes.c_size_t()
    assert lib.cmnn_channel_mean_workspace(g(n=3), 96, ctypes.byref(n)) == 0
    assert n.value == 3 * 65 * 96 * 4  # 64 partial sums and the mean per sample and channel
    assert lib.cmnn_channel_mean_workspace(g(), 288, ctypes.byref(n)) == EINVAL
    assert lib.cmnn_channel_mean_workspace(g(n=1 << 26, d=1, h=1, w=1), 32, ctypes.byref(n)) == EINVAL
    assert lib.cmnn_channel_mean(g(), P, 32, P2, P, 10, NULL) == EINVAL  # workspace too small
    assert lib.cmnn_mse_workspace(0, ctypes.byref(n)) == EINVAL
    assert lib.cmnn_mse_workspace(100, ctypes.byref(n)) == 0
    need = n.value
    mse = lambda c=32, creal=3, wsb=need, ws=P: lib.cmnn_mse(100, P, c, creal, P2, P2, P, NULL, ws, wsb, NULL)
    assert mse(creal=33) == EINVAL
    assert mse(creal=0) == EINVAL
    assert mse(wsb=need - 4) == EINVAL
    assert mse(ws=NULL) == EINVAL
    assert lib.cmnn_clip_grad_norm_workspace(0, ctypes.byref(n)) == EINVAL
    assert lib.cmnn_clip_grad_norm_workspace(1000, ctypes.byref(n)) == 0
    cl = lambda mx, wsb: lib.cmnn_clip_grad_norm(1000, P, ctypes.c_float(mx), P2, P, wsb, NULL)
    assert cl(-1.0, n.value) == EINVAL
    assert cl(float("nan"), n.value) == EINVAL
    assert cl(1.0, n.value - 4) == EINVAL
