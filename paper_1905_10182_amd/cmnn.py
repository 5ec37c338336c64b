"""Python binding of libcmnn (C ABI in include/cmnn.h): argument marshalling
for torch device tensors.  All arithmetic runs in the HIP kernels; the module
raises if the library is missing (no CPU fallback)."""
import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcmnn.so")

OK, EINVAL, EHIP = 0, -1, -3
CALIGN = 32
ACT_NONE, ACT_LEAKY = 0, 1

EXPORTS = ["cmnn_conv3d_fwd", "cmnn_conv3d_bwd_data", "cmnn_conv3d_bwd_data_act", "cmnn_conv3d_bwd_weight_workspace",
           "cmnn_conv3d_bwd_weight", "cmnn_conv3d_bwd_weight_noalloc",
           "cmnn_act_bwd", "cmnn_pool2_fwd", "cmnn_pool2_bwd", "cmnn_up2_fwd", "cmnn_up2_bwd", "cmnn_concat_fwd",
           "cmnn_concat_bwd", "cmnn_up2_concat_fwd", "cmnn_up2_bwd_act", "cmnn_pool2_bwd_add_act",
           "cmnn_add", "cmnn_channel_mean_workspace", "cmnn_channel_mean",
           "cmnn_channel_mean_concat", "cmnn_channel_mean_add_act", "cmnn_mse_workspace",
           "cmnn_mse", "cmnn_clip_grad_norm_workspace", "cmnn_clip_grad_norm", "cmnn_adam", "cmnn_pack_weights",
           "cmnn_pack_channels", "cmnn_unpack_channels", "cmnn_gather_samples", "cmnn_gather_pack_channels",
           "cmnn_pack_weights_batch"]


class Geom(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("d", ctypes.c_int32), ("h", ctypes.c_int32), ("w", ctypes.c_int32),
                ("periodic", ctypes.c_int32 * 3)]


class PackJob(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p), ("w_fwd", ctypes.c_void_p), ("w_t", ctypes.c_void_p),
                ("cin", ctypes.c_int32), ("cout", ctypes.c_int32)]


PACK_MAX = 32


def geom(n, d, h, w, periodic=(1, 0, 1)):
    g = Geom()
    g.n, g.d, g.h, g.w = int(n), int(d), int(h), int(w)
    for a in range(3):
        g.periodic[a] = int(periodic[a])
    return g


class CmnnError(RuntimeError):
    pass


_lib = None


def load_library():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is missing: build it with `python -m paper_1905_10182_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, f32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_float
    G = ctypes.POINTER(Geom)
    lib.cmnn_conv3d_fwd.argtypes = [G, vp, i32, vp, vp, i32, i32, vp, vp]
    lib.cmnn_conv3d_bwd_data.argtypes = [G, vp, i32, vp, i32, vp, vp]
    lib.cmnn_conv3d_bwd_data_act.argtypes = [G, vp, i32, vp, i32, vp, i32, vp, vp]
    lib.cmnn_conv3d_bwd_weight_workspace.argtypes = [G, i32, i32, ctypes.POINTER(sz)]
    lib.cmnn_conv3d_bwd_weight.argtypes = [G, vp, i32, vp, i32, vp, vp, vp, sz, vp]
    lib.cmnn_conv3d_bwd_weight_noalloc.argtypes = [G, vp, i32, vp, i32, vp, vp, vp]
    lib.cmnn_act_bwd.argtypes = [vp, vp, vp, sz, i32, vp]
    for f in (lib.cmnn_pool2_fwd, lib.cmnn_pool2_bwd, lib.cmnn_up2_fwd, lib.cmnn_up2_bwd):
        f.argtypes = [G, vp, i32, vp, vp]
    lib.cmnn_concat_fwd.argtypes = [sz, vp, i32, vp, i32, vp, vp]
    lib.cmnn_concat_bwd.argtypes = [sz, vp, i32, i32, vp, vp, vp]
    lib.cmnn_up2_concat_fwd.argtypes = [G, vp, i32, vp, i32, vp, vp]
    lib.cmnn_up2_bwd_act.argtypes = [G, vp, i32, i32, vp, i32, vp, vp]
    lib.cmnn_pool2_bwd_add_act.argtypes = [G, vp, i32, vp, i32, vp, i32, vp, vp]
    lib.cmnn_add.argtypes = [sz, vp, vp, vp, vp]
    lib.cmnn_channel_mean_workspace.argtypes = [G, i32, ctypes.POINTER(sz)]
    lib.cmnn_channel_mean.argtypes = [G, vp, i32, vp, vp, sz, vp]
    lib.cmnn_channel_mean_concat.argtypes = [G, vp, i32, vp, vp, sz, vp]
    lib.cmnn_channel_mean_add_act.argtypes = [G, vp, i32, i32, vp, i32, vp, i32, vp, vp, sz, vp]
    lib.cmnn_mse_workspace.argtypes = [sz, ctypes.POINTER(sz)]
    lib.cmnn_mse.argtypes = [sz, vp, i32, i32, vp, vp, vp, vp, vp, sz, vp]
    lib.cmnn_clip_grad_norm_workspace.argtypes = [sz, ctypes.POINTER(sz)]
    lib.cmnn_clip_grad_norm.argtypes = [sz, vp, f32, vp, vp, sz, vp]
    lib.cmnn_adam.argtypes = [sz, vp, vp, vp, vp, f32, f32, f32, f32, f32, i32, vp]
    lib.cmnn_pack_weights.argtypes = [vp, i32, i32, vp, vp, vp]
    lib.cmnn_pack_channels.argtypes = [sz, vp, i32, vp, i32, vp]
    lib.cmnn_unpack_channels.argtypes = [sz, vp, i32, vp, i32, vp]
    lib.cmnn_gather_samples.argtypes = [i32, vp, sz, vp, i32, i32, vp, vp]
    lib.cmnn_pack_weights_batch.argtypes = [i32, ctypes.POINTER(PackJob), vp]
    lib.cmnn_gather_pack_channels.argtypes = [i32, vp, sz, vp, i32, i32, vp, i32, vp]
    for name in EXPORTS:
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _s():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(rc, what):
    if rc != OK:
        raise CmnnError(f"{what} failed with status {rc}")


def nvox(g):
    return g.n * g.d * g.h * g.w


def conv_fwd(g, x, cin, w, b, cout, act, y):
    _check(load_library().cmnn_conv3d_fwd(ctypes.byref(g), _p(x), cin, _p(w), _p(b), cout, act, _p(y), _s()),
           "conv3d_fwd")


def conv_bwd_data_act(g, dy, cout, w_t, cin, gate, act, dx):
    """Data gradient with the producing layer's activation gradient fused in:
    dx = conv_bwd_data(dy) times the slope of `act` at its output `gate`."""
    _check(load_library().cmnn_conv3d_bwd_data_act(ctypes.byref(g), _p(dy), cout, _p(w_t), cin, _p(gate), act,
                                                   _p(dx), _s()), "conv3d_bwd_data_act")


def conv_bwd_data(g, dy, cout, w_t, cin, dx):
    _check(load_library().cmnn_conv3d_bwd_data(ctypes.byref(g), _p(dy), cout, _p(w_t), cin, _p(dx), _s()),
           "conv3d_bwd_data")


def conv_bwd_weight_workspace(g, cin, cout):
    n = ctypes.c_size_t()
    _check(load_library().cmnn_conv3d_bwd_weight_workspace(ctypes.byref(g), cin, cout, ctypes.byref(n)),
           "bwd_weight_workspace")
    return n.value


def conv_bwd_weight(g, x, cin, dy, cout, dw, db, ws):
    _check(load_library().cmnn_conv3d_bwd_weight(ctypes.byref(g), _p(x), cin, _p(dy), cout, _p(dw), _p(db), _p(ws),
                                                 ws.numel() * ws.element_size(), _s()), "conv3d_bwd_weight")


def conv_bwd_weight_noalloc(g, x, cin, dy, cout, dw, db):
    """conv_bwd_weight without a workspace (the library's fixed device scratch)."""
    _check(load_library().cmnn_conv3d_bwd_weight_noalloc(ctypes.byref(g), _p(x), cin, _p(dy), cout, _p(dw), _p(db),
                                                         _s()), "conv3d_bwd_weight_noalloc")


def act_bwd(y, dy, dpre, act=ACT_LEAKY):
    _check(load_library().cmnn_act_bwd(_p(y), _p(dy), _p(dpre), y.numel(), act, _s()), "act_bwd")


def pool2_fwd(g, x, c, y):
    _check(load_library().cmnn_pool2_fwd(ctypes.byref(g), _p(x), c, _p(y), _s()), "pool2_fwd")


def pool2_bwd(g, dy, c, dx):
    _check(load_library().cmnn_pool2_bwd(ctypes.byref(g), _p(dy), c, _p(dx), _s()), "pool2_bwd")


def up2_fwd(g, x, c, y):
    _check(load_library().cmnn_up2_fwd(ctypes.byref(g), _p(x), c, _p(y), _s()), "up2_fwd")


def up2_bwd(g, dy, c, dx):
    _check(load_library().cmnn_up2_bwd(ctypes.byref(g), _p(dy), c, _p(dx), _s()), "up2_bwd")


def concat_fwd(nv, a, ca, b, cb, y):
    _check(load_library().cmnn_concat_fwd(nv, _p(a), ca, _p(b), cb, _p(y), _s()), "concat_fwd")


def concat_bwd(nv, dy, ca, cb, da, db):
    _check(load_library().cmnn_concat_bwd(nv, _p(dy), ca, cb, _p(da), _p(db), _s()), "concat_bwd")


def _part(t, off):
    """Pointer to channel `off` of every voxel row of t (a channel part read in place)."""
    return None if t is None else ctypes.c_void_p(t.data_ptr() + off * t.element_size())


def up2_concat_fwd(g, skip, cs, x, cx, y):
    """y = [skip | up2(x)] at the fine level; g is the coarse geometry of x."""
    _check(load_library().cmnn_up2_concat_fwd(ctypes.byref(g), _p(skip), cs, _p(x), cx, _p(y), _s()),
           "up2_concat_fwd")


def up2_bwd_act(g, dy, off, ldy, c, gate, act, dx):
    """dx (coarse) = act'(gate) * up2 gradient of channels [off, off + c) of
    dy (fine, ldy channels per voxel); g is the coarse geometry."""
    _check(load_library().cmnn_up2_bwd_act(ctypes.byref(g), _part(dy, off), ldy, c, _p(gate), act, _p(dx), _s()),
           "up2_bwd_act")


def pool2_bwd_add_act(g, dy, c, skip, off, ldskip, gate, act, dx):
    """dx (fine) = act'(gate) * (pool2 gradient of dy + channels [off, off + c)
    of skip, ldskip channels per voxel; skip None: no term); g is the fine geometry."""
    _check(load_library().cmnn_pool2_bwd_add_act(ctypes.byref(g), _p(dy), c, _part(skip, off), ldskip, _p(gate),
                                                 act, _p(dx), _s()), "pool2_bwd_add_act")


def add(a, b, y):
    _check(load_library().cmnn_add(a.numel(), _p(a), _p(b), _p(y), _s()), "add")


def channel_mean_workspace(g, c):
    n = ctypes.c_size_t()
    _check(load_library().cmnn_channel_mean_workspace(ctypes.byref(g), c, ctypes.byref(n)), "channel_mean_workspace")
    return n.value


def channel_mean(g, x, c, y, ws):
    _check(load_library().cmnn_channel_mean(ctypes.byref(g), _p(x), c, _p(y), _p(ws), ws.numel() * ws.element_size(),
                                            _s()), "channel_mean")


def channel_mean_concat(g, x, c, y, ws):
    """y = [x | per-sample channel means of x, broadcast]."""
    _check(load_library().cmnn_channel_mean_concat(ctypes.byref(g), _p(x), c, _p(y), _p(ws),
                                                   ws.numel() * ws.element_size(), _s()), "channel_mean_concat")


def channel_mean_add_act(g, dy, off, ldy, c, skip, skip_off, ldskip, gate, act, dx, ws):
    """dx = act'(gate) * (channels [skip_off, +c) of skip + the broadcast channel
    means of channels [off, +c) of dy); ldy, ldskip: channels per voxel row."""
    _check(load_library().cmnn_channel_mean_add_act(ctypes.byref(g), _part(dy, off), ldy, c, _part(skip, skip_off),
                                                    ldskip, _p(gate), act, _p(dx), _p(ws),
                                                    ws.numel() * ws.element_size(), _s()), "channel_mean_add_act")


def mse_workspace(nv):
    n = ctypes.c_size_t()
    _check(load_library().cmnn_mse_workspace(nv, ctypes.byref(n)), "mse_workspace")
    return n.value


def mse(nv, pred, c, creal, target, weight, loss2, dpred, ws):
    _check(load_library().cmnn_mse(nv, _p(pred), c, creal, _p(target), _p(weight), _p(loss2), _p(dpred), _p(ws),
                                   ws.numel() * ws.element_size(), _s()), "mse")


def clip_grad_norm_workspace(n):
    k = ctypes.c_size_t()
    _check(load_library().cmnn_clip_grad_norm_workspace(n, ctypes.byref(k)), "clip_grad_norm_workspace")
    return k.value


def clip_grad_norm(g, max_norm, norm_out, ws):
    _check(load_library().cmnn_clip_grad_norm(g.numel(), _p(g), max_norm, _p(norm_out), _p(ws),
                                              ws.numel() * ws.element_size(), _s()), "clip_grad_norm")


def adam(p, g, m, v, lr, b1, b2, eps, wd, step):
    _check(load_library().cmnn_adam(p.numel(), _p(p), _p(g), _p(m), _p(v), lr, b1, b2, eps, wd, step, _s()), "adam")


def pack_weights(w, cin, cout, w_fwd, w_t):
    _check(load_library().cmnn_pack_weights(_p(w), cin, cout, _p(w_fwd), _p(w_t), _s()), "pack_weights")


def pack_jobs(layers):
    """Descriptor array for pack_weights_batch from (w, cin, cout, w_fwd, w_t) tuples."""
    jobs = (PackJob * len(layers))()
    for j, (w, cin, cout, wf, wt) in zip(jobs, layers):
        j.w, j.w_fwd, j.w_t, j.cin, j.cout = w.data_ptr(), wf.data_ptr(), wt.data_ptr(), cin, cout
    return jobs


def pack_weights_batch(jobs):
    _check(load_library().cmnn_pack_weights_batch(len(jobs), jobs, _s()), "pack_weights_batch")


def pack_channels(nv, src, cs, dst, c):
    _check(load_library().cmnn_pack_channels(nv, _p(src), cs, _p(dst), c, _s()), "pack_channels")


def unpack_channels(nv, src, c, dst, cs):
    _check(load_library().cmnn_unpack_channels(nv, _p(src), c, _p(dst), cs, _s()), "unpack_channels")


def gather_samples(idx, src, dst):
    """dst [np][nsel][nvs] = src [np][nsrc][nvs] at samples idx (device int32 [nsel])."""
    np_, nsrc, nvs = src.shape
    _check(load_library().cmnn_gather_samples(idx.numel(), _p(idx), nvs, _p(src), nsrc, np_, _p(dst), _s()),
           "gather_samples")


def gather_pack_channels(idx, src, dst, c):
    """dst BF16 [nsel * nvs][c] = the packed channels of src [cs][nsrc][nvs] at samples idx."""
    cs, nsrc, nvs = src.shape
    _check(load_library().cmnn_gather_pack_channels(idx.numel(), _p(idx), nvs, _p(src), nsrc, cs, _p(dst), c, _s()),
           "gather_pack_channels")
