"""GPU checks of the warm-start network kernels (libcmnn, through the C ABI)
against the FP64 network oracle on BF16-exact inputs.

BF16 x BF16 products are exact in FP32, so the kernels differ from the oracle
only by FP32 accumulation order and the final rounding of BF16 outputs:
BF16 outputs must be within one BF16 ulp (2^-8 relative) of the oracle plus
1e-5 of the accumulated magnitude; FP32 outputs within 1e-5 relative.
"""
import sys

import numpy as np
import pytest

from oracle import conv_oracle as C
import workloads as W

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def nn():
    from paper_1905_10182_amd import cmnn
    cmnn.load_library()
    return cmnn


def bf16_tensor(torch, a):
    """(device BF16 tensor, the same values as float64 numpy)."""
    t = torch.as_tensor(np.asarray(a, np.float32)).to(torch.bfloat16).to("cuda:0")
    return t, t.float().cpu().numpy().astype(np.float64)


def randn(shape, seed, scale=1.0):
    return W.generator(seed).standard_normal(shape) * scale


def close_bf16(got, ref, mag):
    err = np.abs(got - ref)
    bound = np.abs(ref) * 2.0 ** -8 + 1e-5 * mag + 1e-30
    return float((err / bound).max())


# the first three take the generic kernel (extents not multiples of the 4 x 4 x 16 brick),
# the rest the brick-tiled one: several bricks with periodic, zero and mixed padding, a single
# brick that wraps onto itself, and every output-tile width (16 * NB for NB = 2, 4, 6)
SHAPES = [((2, 3, 5, 7), 32, 64, (1, 0, 1)), ((1, 4, 6, 8), 64, 32, (0, 1, 0)), ((1, 2, 4, 6), 32, 96, (1, 1, 1)),
          ((2, 4, 8, 32), 32, 64, (1, 0, 1)), ((1, 8, 4, 16), 96, 32, (0, 1, 0)), ((1, 4, 4, 16), 64, 96, (1, 1, 1)),
          ((2, 4, 4, 16), 32, 160, (1, 0, 1)), ((1, 4, 8, 16), 192, 64, (0, 0, 0))]


@pytest.mark.parametrize("dims,cin,cout,per", SHAPES)
def test_conv_forward(torch, nn, dims, cin, cout, per):
    log(f"conv fwd {dims} {cin}->{cout} periodic={per}")
    g = nn.geom(*dims, periodic=per)
    x, xr = bf16_tensor(torch, randn(dims + (cin,), 1))
    w, wr = bf16_tensor(torch, randn((27, cout, cin), 2, 0.1))
    b = torch.as_tensor(randn((cout,), 3, 0.1), dtype=torch.float32, device="cuda:0")
    for act in (nn.ACT_NONE, nn.ACT_LEAKY):
        y = torch.empty(dims + (cout,), dtype=torch.bfloat16, device="cuda:0")
        nn.conv_fwd(g, x, cin, w, b, cout, act, y)
        ref = C.conv3d(xr, wr, b.cpu().numpy().astype(np.float64), per)
        if act == nn.ACT_LEAKY:
            ref = C.leaky(ref)
        mag = C.conv3d(np.abs(xr), np.abs(wr), None, per)
        r = close_bf16(y.float().cpu().numpy(), ref, mag)
        log(f"  act={act}: max error / bound = {r:.3f}")
        assert r <= 1.0


@pytest.mark.parametrize("dims,cin,cout,per", SHAPES)
def test_conv_backward(torch, nn, dims, cin, cout, per):
    log(f"conv bwd {dims} {cin}->{cout} periodic={per}")
    g = nn.geom(*dims, periodic=per)
    x, xr = bf16_tensor(torch, randn(dims + (cin,), 4))
    wm = torch.as_tensor(randn((27, cout, cin), 5, 0.1), dtype=torch.float32, device="cuda:0")
    wf = torch.empty((27, cout, cin), dtype=torch.bfloat16, device="cuda:0")
    wt = torch.empty((27, cin, cout), dtype=torch.bfloat16, device="cuda:0")
    nn.pack_weights(wm, cin, cout, wf, wt)
    wr = wf.float().cpu().numpy().astype(np.float64)
    assert np.array_equal(wt.float().cpu().numpy(), wf.float().cpu().numpy().transpose(0, 2, 1))
    dy, dyr = bf16_tensor(torch, randn(dims + (cout,), 6))
    dx = torch.empty(dims + (cin,), dtype=torch.bfloat16, device="cuda:0")
    nn.conv_bwd_data(g, dy, cout, wt, cin, dx)
    rdx, rdw, rdb = C.conv3d_grads(xr, wr, dyr, per)
    magx, _, _ = C.conv3d_grads(np.abs(xr), np.abs(wr), np.abs(dyr), per)
    r = close_bf16(dx.float().cpu().numpy(), rdx, magx)
    log(f"  dx: max error / bound = {r:.3f}")
    assert r <= 1.0
    # the same with the producing layer's activation gradient fused in: gate is
    # that layer's leaky-ReLU output (mixed signs, some exact zeros)
    gv = randn(dims + (cin,), 9)
    gv[np.abs(gv) < 0.1] = 0.0
    gate, gr = bf16_tensor(torch, gv)
    dxa = torch.empty_like(dx)
    nn.conv_bwd_data_act(g, dy, cout, wt, cin, gate, nn.ACT_LEAKY, dxa)
    rdxa = C.leaky_grad_from_output(gr, rdx)
    magxa = C.leaky_grad_from_output(gr, magx)
    r = close_bf16(dxa.float().cpu().numpy(), rdxa, magxa)
    log(f"  dx with the activation gradient: max error / bound = {r:.3f}")
    assert r <= 1.0
    nn.conv_bwd_data_act(g, dy, cout, wt, cin, gate, nn.ACT_NONE, dxa)
    assert torch.equal(dxa, dx)  # no activation: the plain data gradient, bitwise
    ws = torch.empty(nn.conv_bwd_weight_workspace(g, cin, cout) // 4, dtype=torch.float32, device="cuda:0")
    dw = torch.empty((27, cout, cin), dtype=torch.float32, device="cuda:0")
    db = torch.empty((cout,), dtype=torch.float32, device="cuda:0")
    nn.conv_bwd_weight(g, x, cin, dy, cout, dw, db, ws)
    e_w = np.linalg.norm(dw.cpu().numpy() - rdw) / np.linalg.norm(rdw)
    e_b = np.linalg.norm(db.cpu().numpy() - rdb) / np.linalg.norm(rdb)
    log(f"  dw rel {e_w:.2e}  db rel {e_b:.2e}")
    assert e_w < 1e-5 and e_b < 1e-5
    dw2 = torch.empty_like(dw)
    nn.conv_bwd_weight(g, x, cin, dy, cout, dw2, None, ws)
    assert torch.equal(dw, dw2)  # deterministic


LARGE = [("fwd", (4, 32, 32, 64), 96, 32, (1, 0, 1)),    # brick kernel, 16-channel-pair tiles (NB = 2)
         ("fwd", (16, 16, 16, 32), 64, 96, (1, 0, 1)),   # 512 bricks: 96-wide tiles (NB = 6)
         ("fwd", (16, 16, 16, 32), 32, 64, (0, 1, 1)),   # 64-wide tiles (NB = 4)
         ("bwd", (16, 16, 16, 32), 96, 64, (1, 0, 1)),   # data gradient with 96 outputs (NB = 6)
         ("bwd", (16, 16, 16, 32), 64, 32, (1, 1, 0))]   # data gradient with 64 outputs (NB = 4)


@pytest.mark.parametrize("kind,dims,cin,cout,per", LARGE)
def test_conv_large_sampled(torch, nn, kind, dims, cin, cout, per):
    """Warm-start-sized levels in the launch configurations training uses,
    checked on 64 sampled output voxels computed directly from the definition
    (forward: sum over taps of w[t] x[v + off]; data gradient: sum over taps of
    w[t]^T dy[v - off], zero padding where the shifted voxel leaves a
    non-periodic axis)."""
    log(f"conv {kind} sampled {dims} layer {cin}->{cout} periodic={per}")
    g = nn.geom(*dims, periodic=per)
    cx, cy = (cin, cout) if kind == "fwd" else (cout, cin)  # input / output channels of the launch
    x, xr = bf16_tensor(torch, randn(dims + (cx,), 7))
    w, wr = bf16_tensor(torch, randn((27, cout, cin), 8, 0.05))
    y = torch.empty(dims + (cy,), dtype=torch.bfloat16, device="cuda:0")
    if kind == "fwd":
        nn.conv_fwd(g, x, cin, w, None, cout, nn.ACT_NONE, y)
        sign, wmat = 1, wr  # y = w[t] @ x
    else:
        wt = torch.empty((27, cin, cout), dtype=torch.bfloat16, device="cuda:0")
        wt.copy_(w.transpose(1, 2))
        nn.conv_bwd_data(g, x, cout, wt, cin, y)
        sign, wmat = -1, wr.transpose(0, 2, 1)  # dx = w[t]^T @ dy
    yg = y.float().cpu().numpy()
    gen = W.generator(9)
    for _ in range(64):
        v = [int(gen.integers(s_)) for s_ in dims]
        acc = np.zeros(cy)
        for t, off in enumerate(C.taps()):
            src, ok = [v[0]], True
            for a in range(3):
                q = v[a + 1] + sign * off[a]
                if not 0 <= q < dims[a + 1]:
                    if not per[a]:
                        ok = False
                        break
                    q %= dims[a + 1]
                src.append(q)
            if ok:
                acc += wmat[t] @ xr[tuple(src)]
        assert np.all(np.abs(yg[tuple(v)] - acc) <= np.abs(acc) * 2.0 ** -8 + 1e-3), (v, kind)


def test_conv_past_4_gib_tensors(torch, nn):
    """Convolutions on activations of more than 4 GiB (16 x 64 x 256 x 272
    voxels, 32 channels, 4.6 GB per tensor): the forward and data-gradient
    brick tiles on 64 sampled output voxels from the definition, and the
    weight gradient (which takes its generic kernel past 2^32 bytes) through
    the adjoint identity sum_v dy . conv(x, w) = sum w . dW(x, dy), exact up
    to the BF16 rounding of the forward output."""
    dims, cin, cout, per = (16, 64, 256, 272), 32, 32, (1, 0, 1)
    nv = int(np.prod(dims))
    assert nv * cin * 2 >= 2 ** 32
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < 40 * 2 ** 30:
        pytest.skip(f"needs 40 GiB of free device memory, {free / 2**30:.0f} GiB free")
    log(f"conv past 4 GiB: {dims} {cin}->{cout}")
    dev, bf = "cuda:0", torch.bfloat16
    gen = torch.Generator(device=dev)
    gen.manual_seed(36)
    g = nn.geom(*dims, periodic=per)
    x = torch.randn(dims + (cin,), generator=gen, device=dev).to(bf)
    dy = torch.randn(dims + (cout,), generator=gen, device=dev).to(bf)
    w, wr = bf16_tensor(torch, randn((27, cout, cin), 37, 0.05))
    wt = w.transpose(1, 2).contiguous()
    y = torch.empty(dims + (cout,), dtype=bf, device=dev)
    dx = torch.empty(dims + (cin,), dtype=bf, device=dev)
    nn.conv_fwd(g, x, cin, w, None, cout, nn.ACT_NONE, y)
    nn.conv_bwd_data(g, dy, cout, wt, cin, dx)
    rg = W.generator(38)
    for kind, src_t, out_t, sign, wmat in (("fwd", x, y, 1, wr), ("bwd", dy, dx, -1, wr.transpose(0, 2, 1))):
        for _ in range(64):
            v = [int(rg.integers(s_)) for s_ in dims]
            acc = np.zeros(out_t.shape[-1])
            for t, off in enumerate(C.taps()):
                srcv, ok = [v[0]], True
                for a in range(3):
                    q = v[a + 1] + sign * off[a]
                    if not 0 <= q < dims[a + 1]:
                        if not per[a]:
                            ok = False
                            break
                        q %= dims[a + 1]
                    srcv.append(q)
                if ok:
                    acc += wmat[t] @ src_t[tuple(srcv)].double().cpu().numpy()
            got = out_t[tuple(v)].double().cpu().numpy()
            assert np.all(np.abs(got - acc) <= np.abs(acc) * 2.0 ** -8 + 1e-3), (v, kind)
    del dx
    ws = torch.empty(nn.conv_bwd_weight_workspace(g, cin, cout) // 4, dtype=torch.float32, device=dev)
    dw = torch.empty((27, cout, cin), dtype=torch.float32, device=dev)
    nn.conv_bwd_weight(g, x, cin, dy, cout, dw, None, ws)
    prod = dy.double() * y.double()
    lhs, rms = float(prod.sum().item()), float(prod.square().sum().sqrt().item())
    del prod
    rhs = float((w.double() * dw.double()).sum().item())
    # the forward output's BF16 rounding (<= 2^-9 relative, random in sign)
    # moves <dy, y> by about 2^-9 rms; one missing tap would move <w, dW> by
    # about 0.05 x 32 x sqrt(voxels), over ten times more
    log(f"  <dy, y> = {lhs:.6e}, <w, dW> = {rhs:.6e}, rounding scale {2.0 ** -9 * rms:.3e}")
    assert abs(lhs - rhs) <= 2.0 ** -6 * rms
    del x, dy, y, ws, dw
    torch.cuda.empty_cache()


@pytest.mark.parametrize("c,ca,cb,nl", [(32, 32, 64, 1000), (12, 12, 20, 1001)])
def test_elementwise_ops(torch, nn, c, ca, cb, nl):
    """Channel counts that are multiples of 8 take the 16-byte kernels, the others the scalar ones."""
    log(f"pool / upsample / concat / add / act_bwd c={c} concat {ca}+{cb} n={nl}")
    dims = (2, 4, 6, 8)
    g = nn.geom(*dims)
    gc = nn.geom(2, 2, 3, 4)
    x, xr = bf16_tensor(torch, randn(dims + (c,), 10))
    y = torch.empty((2, 2, 3, 4, c), dtype=torch.bfloat16, device="cuda:0")
    nn.pool2_fwd(g, x, c, y)
    assert close_bf16(y.float().cpu().numpy(), C.pool2(xr), np.abs(C.pool2(np.abs(xr)))) <= 1.0
    dy, dyr = bf16_tensor(torch, randn((2, 2, 3, 4, c), 11))
    dx = torch.empty(dims + (c,), dtype=torch.bfloat16, device="cuda:0")
    nn.pool2_bwd(g, dy, c, dx)
    assert np.array_equal(dx.float().cpu().numpy(), C.pool2_grad(dyr))  # exact: division by 8
    u = torch.empty(dims + (c,), dtype=torch.bfloat16, device="cuda:0")
    nn.up2_fwd(gc, dy, c, u)
    assert np.array_equal(u.float().cpu().numpy(), C.up2(dyr))
    du = torch.empty((2, 2, 3, 4, c), dtype=torch.bfloat16, device="cuda:0")
    nn.up2_bwd(gc, x, c, du)
    assert close_bf16(du.float().cpu().numpy(), C.up2_grad(xr), C.up2_grad(np.abs(xr))) <= 1.0
    a, ar = bf16_tensor(torch, randn((30, ca), 12))
    b, br = bf16_tensor(torch, randn((30, cb), 13))
    cat = torch.empty((30, ca + cb), dtype=torch.bfloat16, device="cuda:0")
    nn.concat_fwd(30, a, ca, b, cb, cat)
    assert np.array_equal(cat.float().cpu().numpy(), np.concatenate([ar, br], 1))
    da = torch.empty_like(a)
    db = torch.empty_like(b)
    nn.concat_bwd(30, cat, ca, cb, da, db)
    assert torch.equal(da, a) and torch.equal(db, b)
    s = torch.empty_like(a)
    nn.add(a, a, s)
    assert torch.equal(s.float(), 2 * a.float())
    yl, ylr = bf16_tensor(torch, randn((nl,), 14))
    gl, glr = bf16_tensor(torch, randn((nl,), 15))
    sl = torch.empty_like(yl)
    nn.add(yl, gl, sl)
    assert close_bf16(sl.float().cpu().numpy(), ylr + glr, np.abs(ylr) + np.abs(glr)) <= 1.0
    out = torch.empty_like(yl)
    nn.act_bwd(yl, gl, out)
    assert close_bf16(out.float().cpu().numpy(), C.leaky_grad_from_output(ylr, glr), np.abs(glr)) <= 1.0


@pytest.mark.parametrize("cs,cx", [(32, 64), (64, 96)])
def test_skip_joins(torch, nn, cs, cx):
    """The U-Net's fused skip joins against the oracle's separate steps
    (upsampling or pooling, concatenation, sum, activation gradient); the
    concatenation's gradient is read in place through its channel stride."""
    log(f"skip joins cs={cs} cx={cx}")
    fine, coarse, ct = (2, 4, 6, 8), (2, 2, 3, 4), cs + cx
    g, gc = nn.geom(*fine), nn.geom(*coarse)
    bf = dict(dtype=torch.bfloat16, device="cuda:0")
    skip, skr = bf16_tensor(torch, randn(fine + (cs,), 40))
    x, xr = bf16_tensor(torch, randn(coarse + (cx,), 41))
    y = torch.full(fine + (ct,), 7.0, **bf)
    nn.up2_concat_fwd(gc, skip, cs, x, cx, y)
    assert np.array_equal(y.float().cpu().numpy(), np.concatenate([skr, C.up2(xr)], -1))
    dcat, dcr = bf16_tensor(torch, randn(fine + (ct,), 42))
    gate_c, gcr = bf16_tensor(torch, randn(coarse + (cx,), 43))
    for act in (nn.ACT_LEAKY, nn.ACT_NONE):
        dx = torch.full(coarse + (cx,), 7.0, **bf)
        nn.up2_bwd_act(gc, dcat, cs, ct, cx, gate_c, act, dx)
        ref = C.up2_grad(dcr[..., cs:])
        if act == nn.ACT_LEAKY:
            ref = C.leaky_grad_from_output(gcr, ref)
        assert close_bf16(dx.float().cpu().numpy(), ref, C.up2_grad(np.abs(dcr[..., cs:]))) <= 1.0, act
    dp, dpr = bf16_tensor(torch, randn(coarse + (cs,), 44))
    gate_f, gfr = bf16_tensor(torch, randn(fine + (cs,), 45))
    for act, with_skip in ((nn.ACT_LEAKY, True), (nn.ACT_NONE, True), (nn.ACT_LEAKY, False)):
        ds = torch.full(fine + (cs,), 7.0, **bf)
        nn.pool2_bwd_add_act(g, dp, cs, dcat if with_skip else None, 0, ct, gate_f, act, ds)
        ref = C.pool2_grad(dpr) + (dcr[..., :cs] if with_skip else 0.0)
        mag = C.pool2_grad(np.abs(dpr)) + (np.abs(dcr[..., :cs]) if with_skip else 0.0)
        if act == nn.ACT_LEAKY:
            ref = C.leaky_grad_from_output(gfr, ref)
        assert close_bf16(ds.float().cpu().numpy(), ref, mag) <= 1.0, (act, with_skip)


def test_joins_past_2_to_32_elements(torch, nn):
    """The skip joins and pooling on tensors of more than 2^32 elements (their
    64-bit index variants; 2 x 256 x 256 x 520 fine voxels, 64 channels): the
    outputs at 2048 sampled voxels against the oracle's operations on each
    voxel's neighbourhood (a concatenation bitwise, sums within a BF16 ulp)."""
    fine, coarse = (2, 256, 256, 520), (2, 128, 128, 260)
    nf = int(np.prod(fine))
    assert nf * 64 >= 2 ** 32
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < 40 * 2 ** 30:
        pytest.skip(f"needs 40 GiB of free device memory, {free / 2**30:.0f} GiB free")
    log("joins past 2^32 elements")
    dev, bf = "cuda:0", torch.bfloat16
    gen = torch.Generator(device=dev)
    gen.manual_seed(32)
    g, gc = nn.geom(*fine), nn.geom(*coarse)
    skip = torch.randn(fine + (32,), generator=gen, device=dev).to(bf)
    x = torch.randn(coarse + (32,), generator=gen, device=dev).to(bf)
    y = torch.empty(fine + (64,), dtype=bf, device=dev)
    nn.up2_concat_fwd(gc, skip, 32, x, 32, y)
    rg = W.generator(33)
    v = np.stack([rg.integers(0, e, 2048) for e in fine], 1)  # (n, d, h, w) of sampled fine voxels
    vc = np.stack([rg.integers(0, e, 2048) for e in coarse], 1)

    def at(t, idx):  # values of t (5-D) at rows of (n, d, h, w) indices, FP64
        i = [torch.as_tensor(idx[:, a], device=dev) for a in range(4)]
        return t[i[0], i[1], i[2], i[3]].double().cpu().numpy()

    par = v.copy()
    par[:, 1:] //= 2
    assert np.array_equal(at(y, v), np.concatenate([at(skip, v), at(x, par)], 1))
    kids = [vc * np.array([1, 2, 2, 2]) + np.array([0, k >> 2, (k >> 1) & 1, k & 1]) for k in range(8)]
    # upsampled part of the concatenation's gradient (y as dy), with the activation gradient
    gate_c = torch.randn(coarse + (32,), generator=gen, device=dev).to(bf)
    dxc = torch.empty(coarse + (32,), dtype=bf, device=dev)
    nn.up2_bwd_act(gc, y, 32, 64, 32, gate_c, nn.ACT_LEAKY, dxc)
    blk = np.stack([at(y, kv)[:, 32:] for kv in kids], 1).reshape(-1, 2, 2, 2, 32)[:, None]  # (s, 1, 2, 2, 2, c)
    ref = np.stack([C.up2_grad(b[None])[0, 0, 0, 0] for b in blk[:, 0]])
    ref = C.leaky_grad_from_output(at(gate_c, vc), ref)
    mag = np.stack([C.up2_grad(np.abs(b[None]))[0, 0, 0, 0] for b in blk[:, 0]])
    assert close_bf16(at(dxc, vc), ref, mag) <= 1.0
    # pooling of the 64-channel tensor
    pc = torch.empty(coarse + (64,), dtype=bf, device=dev)
    nn.pool2_fwd(g, y, 64, pc)
    blk = np.stack([at(y, kv) for kv in kids], 1).reshape(-1, 2, 2, 2, 64)
    ref = np.stack([C.pool2(b[None])[0, 0, 0, 0] for b in blk])
    mag = np.stack([C.pool2(np.abs(b[None]))[0, 0, 0, 0] for b in blk])
    assert close_bf16(at(pc, vc), ref, mag) <= 1.0
    del pc, dxc
    # encoder join: pooling gradient of a coarse 32-channel dy plus the skip part of y, activation gradient at skip
    dyc = torch.randn(coarse + (32,), generator=gen, device=dev).to(bf)
    dxf = torch.empty(fine + (32,), dtype=bf, device=dev)
    nn.pool2_bwd_add_act(g, dyc, 32, y, 0, 64, skip, nn.ACT_LEAKY, dxf)
    ref = C.leaky_grad_from_output(at(skip, v), at(dyc, par) / 8.0 + at(y, v)[:, :32])
    mag = np.abs(at(dyc, par)) / 8.0 + np.abs(at(y, v)[:, :32])
    assert close_bf16(at(dxf, v), ref, mag) <= 1.0
    del skip, x, y, gate_c, dyc, dxf
    torch.cuda.empty_cache()


def test_mse_and_gather_past_2_to_32_elements(torch, nn):
    """The minibatch gather-and-pack and the MSE gradient on more than 2^32
    output elements (their 64-bit index variants): 2 samples of 67,174,400
    voxels packed to 32 channels, and the masked MSE over those voxels; sampled
    voxels against the definitions (the packing's FP32 -> BF16 rounding
    bitwise, the gradient within a BF16 ulp of 2 w (p - t) / (creal sum w))."""
    nvs, nsel, nsrc, c = 67_174_400, 2, 3, 32
    assert nsel * nvs * c >= 2 ** 32
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < 40 * 2 ** 30:
        pytest.skip(f"needs 40 GiB of free device memory, {free / 2**30:.0f} GiB free")
    log("gather + mse past 2^32 elements")
    dev = "cuda:0"
    gen = torch.Generator(device=dev)
    gen.manual_seed(34)
    src = torch.rand((2, nsrc, nvs), generator=gen, device=dev)
    idx = torch.as_tensor([2, 0], dtype=torch.int32, device=dev)
    packed = torch.empty((nsel * nvs, c), dtype=torch.bfloat16, device=dev)
    nn.gather_pack_channels(idx, src, packed, c)
    rg = W.generator(35)
    rows = rg.integers(0, nsel * nvs, 2048)
    rt = torch.as_tensor(rows, device=dev)
    got = packed[rt].float().cpu().numpy()
    b, vv = rows // nvs, rows % nvs
    want = np.stack([src[:, [2, 0][k], int(u)].cpu().numpy() for k, u in zip(b, vv)])
    want = torch.as_tensor(want).to(torch.bfloat16).float().numpy()
    assert np.array_equal(got[:, :2], want) and np.all(got[:, 2:] == 0)
    del src
    nv, creal = nsel * nvs, 3
    tgt = torch.rand((creal, nv), generator=gen, device=dev)
    wt = (torch.rand((nv,), generator=gen, device=dev) > 0.2).float()
    loss = torch.empty(2, dtype=torch.float32, device=dev)
    dpred = torch.empty_like(packed)
    ws = torch.empty(nn.mse_workspace(nv) // 4, dtype=torch.float32, device=dev)
    nn.mse(nv, packed, c, creal, tgt, wt, loss, dpred, ws)
    norm = float(loss[1].item())
    assert abs(norm / (creal * float(wt.double().sum().item())) - 1) < 1e-6
    p = packed[rt].double().cpu().numpy()[:, :creal]
    t = tgt[:, rt].double().cpu().numpy().T
    w = wt[rt].double().cpu().numpy()[:, None]
    ref = 2.0 * w * (p - t) / norm
    g = dpred[rt].float().cpu().numpy()
    assert close_bf16(g[:, :creal], ref, np.abs(ref)) <= 1.0 and np.all(g[:, creal:] == 0)
    del packed, tgt, wt, dpred, ws
    torch.cuda.empty_cache()


@pytest.mark.parametrize("c", [64, 12])
def test_channel_mean(torch, nn, c):
    log(f"channel mean broadcast c={c}")
    dims = (3, 4, 6, 10)
    g = nn.geom(*dims)
    x, xr = bf16_tensor(torch, randn(dims + (c,), 30))
    y = torch.empty_like(x)
    ws = torch.empty(nn.channel_mean_workspace(g, c) // 4, dtype=torch.float32, device="cuda:0")
    nn.channel_mean(g, x, c, y, ws)
    ref = C.channel_mean(xr)
    assert close_bf16(y.float().cpu().numpy(), ref, C.channel_mean(np.abs(xr))) <= 1.0


def test_bottleneck_joins(torch, nn):
    """The global-context join: [x | channel means] bitwise as the separate
    mean and concatenation, and its gradient (mean map self-adjoint, both parts
    of the concatenation's gradient read in place) against the oracle."""
    log("bottleneck joins c=64")
    dims, c = (3, 4, 6, 10), 64
    g = nn.geom(*dims)
    bf = dict(dtype=torch.bfloat16, device="cuda:0")
    ws = torch.empty(nn.channel_mean_workspace(g, c) // 4, dtype=torch.float32, device="cuda:0")
    x, xr = bf16_tensor(torch, randn(dims + (c,), 31))
    gm = torch.empty_like(x)
    nn.channel_mean(g, x, c, gm, ws)
    ref = torch.empty(dims + (2 * c,), **bf)
    nn.concat_fwd(nn.nvox(g), x, c, gm, c, ref)
    y = torch.full(dims + (2 * c,), 7.0, **bf)
    nn.channel_mean_concat(g, x, c, y, ws)
    assert torch.equal(y, ref)
    dcat, dcr = bf16_tensor(torch, randn(dims + (2 * c,), 32))
    for act in (nn.ACT_LEAKY, nn.ACT_NONE):
        dx = torch.full(dims + (c,), 7.0, **bf)
        nn.channel_mean_add_act(g, dcat, c, 2 * c, c, dcat, 0, 2 * c, x, act, dx, ws)
        r = dcr[..., :c] + C.channel_mean(dcr[..., c:])
        if act == nn.ACT_LEAKY:
            r = C.leaky_grad_from_output(xr, r)
        mag = np.abs(dcr[..., :c]) + C.channel_mean(np.abs(dcr[..., c:]))
        assert close_bf16(dx.float().cpu().numpy(), r, mag) <= 1.0, act


def test_clip_grad_norm(torch, nn):
    log("gradient-norm clipping")
    g64 = randn((100003,), 31)
    n = int(g64.size)
    ws = torch.empty(nn.clip_grad_norm_workspace(n) // 4, dtype=torch.float32, device="cuda:0")
    out = torch.empty(2, dtype=torch.float32, device="cuda:0")
    for frac in (0.3, 2.0, 0.0):
        g32 = g64.astype(np.float32)
        ref, norm = C.clip_grad_norm(g32.astype(np.float64), frac * np.linalg.norm(g32.astype(np.float64)))
        g = torch.as_tensor(g32, device="cuda:0")
        nn.clip_grad_norm(g, float(frac * norm), out, ws)
        assert abs(out[0].item() / norm - 1) < 1e-5
        np.testing.assert_allclose(g.cpu().numpy(), ref, rtol=2e-5, atol=1e-7 * np.abs(ref).max())
    g = torch.as_tensor(g64.astype(np.float32), device="cuda:0")
    g[7] = float("inf")
    nn.clip_grad_norm(g, 1.0, out, ws)
    assert out[1].item() == 0.0 and not g.abs().max().item()


@pytest.mark.parametrize("c,creal", [(32, 3), (32, 11), (12, 3)])
def test_masked_mse(torch, nn, c, creal):
    """16-byte gradient kernel (c a multiple of 8, creal inside one or two
    8-channel groups) and the scalar one (c = 12)."""
    log(f"mse c={c} creal={creal}")
    nv = 5000
    p, pr = bf16_tensor(torch, randn((nv, c), 16))
    tgt = torch.as_tensor(randn((creal, nv), 17), dtype=torch.float32, device="cuda:0")
    wt = torch.as_tensor((randn((nv,), 18) > -0.5).astype(np.float32), device="cuda:0")
    loss = torch.empty(2, dtype=torch.float32, device="cuda:0")
    dp = torch.full_like(p, 7.0)
    ws = torch.empty(nn.mse_workspace(nv) // 4, dtype=torch.float32, device="cuda:0")
    nn.mse(nv, p, c, creal, tgt, wt, loss, dp, ws)
    rl, rg = C.mse(pr[:, :creal], tgt.cpu().numpy().astype(np.float64), wt.cpu().numpy().astype(np.float64))
    assert abs(loss[0].item() / rl - 1) < 1e-5
    got = dp.float().cpu().numpy()
    assert close_bf16(got[:, :creal], rg, np.abs(rg)) <= 1.0
    assert np.all(got[:, creal:] == 0)


def test_minibatch_gathers(torch, nn):
    """Gathers of samples from plane-major data: exact copies (FP32) or the
    FP32 -> BF16 rounding of the packing; an out-of-range index gives zeros."""
    log("minibatch gathers")
    nsrc, nvs = 7, 24
    dev = "cuda:0"
    src = torch.as_tensor(randn((3, nsrc, nvs), 22), dtype=torch.float32, device=dev)
    for idx in ([4, 0, 6], [2, 9, -1, 5]):
        ii = torch.as_tensor(idx, dtype=torch.int32, device=dev)
        ok = np.array([0 <= k < nsrc for k in idx])
        ref = np.zeros((3, len(idx), nvs), np.float32)
        ref[:, ok] = src.cpu().numpy()[:, np.array(idx)[ok]]
        for n_vs in (nvs, nvs - 1):  # 4-wide and scalar kernels
            s = src[..., :n_vs].contiguous()
            out = torch.full((3, len(idx), n_vs), 7.0, dtype=torch.float32, device=dev)
            nn.gather_samples(ii, s, out)
            assert np.array_equal(out.cpu().numpy(), ref[..., :n_vs])
        packed = torch.full((len(idx) * nvs, 16), 7.0, dtype=torch.bfloat16, device=dev)
        nn.gather_pack_channels(ii, src[:2].contiguous(), packed, 16)
        want = torch.as_tensor(ref[:2].reshape(2, -1).T).to(torch.bfloat16).float().numpy()
        got = packed.float().cpu().numpy()
        assert np.array_equal(got[:, :2], want) and np.all(got[:, 2:] == 0)


def test_pack_weights_batch(torch, nn):
    """One launch for several layers, bitwise the per-layer packing."""
    log("batched weight packing")
    shapes = [(32, 32), (64, 96), (192, 96), (32, 160)]
    dev = "cuda:0"
    ws = [torch.as_tensor(randn((27, co, ci), 50 + k), dtype=torch.float32, device=dev)
          for k, (ci, co) in enumerate(shapes)]
    outs = [(torch.empty((27, co, ci), dtype=torch.bfloat16, device=dev),
             torch.empty((27, ci, co), dtype=torch.bfloat16, device=dev)) for ci, co in shapes]
    nn.pack_weights_batch(nn.pack_jobs([(w, ci, co, wf, wt) for w, (ci, co), (wf, wt) in zip(ws, shapes, outs)]))
    for w, (ci, co), (wf, wt) in zip(ws, shapes, outs):
        rf, rt = torch.empty_like(wf), torch.empty_like(wt)
        nn.pack_weights(w, ci, co, rf, rt)
        assert torch.equal(wf, rf) and torch.equal(wt, rt)
        assert torch.equal(wt, w.to(torch.bfloat16).transpose(1, 2))


def test_mse_adam_and_channel_packing(torch, nn):
    log("mse / adam / pack channels")
    nv, c, creal = 5000, 32, 3
    p, pr = bf16_tensor(torch, randn((nv, c), 16))
    tgt = torch.as_tensor(randn((creal, nv), 17), dtype=torch.float32, device="cuda:0")
    wt = torch.as_tensor((randn((nv,), 18) > -0.5).astype(np.float32), device="cuda:0")
    loss = torch.empty(2, dtype=torch.float32, device="cuda:0")
    dp = torch.empty_like(p)
    ws = torch.empty(nn.mse_workspace(nv) // 4, dtype=torch.float32, device="cuda:0")
    nn.mse(nv, p, c, creal, tgt, wt, loss, dp, ws)
    rl, rg = C.mse(pr, tgt.cpu().numpy().astype(np.float64), wt.cpu().numpy().astype(np.float64))
    assert abs(loss[0].item() / rl - 1) < 1e-5
    assert close_bf16(dp.float().cpu().numpy(), rg, np.abs(rg)) <= 1.0
    n = 777
    pm = torch.as_tensor(randn((n,), 19), dtype=torch.float32, device="cuda:0")
    gm = torch.as_tensor(randn((n,), 20), dtype=torch.float32, device="cuda:0")
    m = torch.zeros_like(pm)
    v = torch.zeros_like(pm)
    ref_p, ref_m, ref_v = pm.cpu().numpy().astype(np.float64), np.zeros(n), np.zeros(n)
    g64 = gm.cpu().numpy().astype(np.float64)
    for step in (1, 2, 3):
        nn.adam(pm, gm, m, v, 1e-3, 0.9, 0.999, 1e-8, 1e-4, step)
        ref_p, ref_m, ref_v = C.adam(ref_p, g64, ref_m, ref_v, 1e-3, 0.9, 0.999, 1e-8, 1e-4, step)
    np.testing.assert_allclose(pm.cpu().numpy(), ref_p, rtol=0, atol=1e-6)
    src = torch.as_tensor(randn((2, 100), 21), dtype=torch.float32, device="cuda:0")
    packed = torch.empty((100, 32), dtype=torch.bfloat16, device="cuda:0")
    nn.pack_channels(100, src, 2, packed, 32)
    assert np.array_equal(packed.float().cpu().numpy()[:, :2], src.to(torch.bfloat16).float().cpu().numpy().T)
    assert np.all(packed.float().cpu().numpy()[:, 2:] == 0)
    back = torch.empty((2, 100), dtype=torch.float32, device="cuda:0")
    nn.unpack_channels(100, packed, 32, back, 2)
    assert torch.equal(back, src.to(torch.bfloat16).float())
    packed12 = torch.full((100, 12), 7.0, dtype=torch.bfloat16, device="cuda:0")  # the scalar packing kernel
    nn.pack_channels(100, src, 2, packed12, 12)
    assert torch.equal(packed12[:, :2], packed[:, :2]) and np.all(packed12.float().cpu().numpy()[:, 2:] == 0)
