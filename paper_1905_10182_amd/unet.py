"""3D convolutional U-Net on the libcmnn kernels (BF16 MFMA convolutions).

The network maps per-voxel inputs of a forced channel (fluid mask, wall-
distance feature) to the normalised steady velocity.  Every arithmetic step
runs in libcmnn; PyTorch only allocates the tensors.  Layout NDHWC BF16 with
channels padded to 32; padding is periodic in z and x, zero in y (the walls).

Architecture (widths w0, w1, w2; leaky ReLU after every 3x3x3 convolution
except the head; the channel means at the bottleneck give every voxel the
sample-wide context, e.g. the total blockage that sets the flow rate):

    enc0: conv(in -> w0), conv(w0 -> w0)              full resolution  -> s0
    enc1: pool, conv(w0 -> w1), conv(w1 -> w1)         1/2              -> s1
    mid:  pool, conv(w1 -> w2), concat(per-sample channel means),
          conv(2 w2 -> w2)                             1/4
    dec1: up, concat(s1), conv(w1 + w2 -> w1), conv(w1 -> w1)
    dec0: up, concat(s0), conv(w0 + w1 -> w0), conv(w0 -> w0)
    head: conv(w0 -> out)
"""
import numpy as np

from . import cmnn

PERIODIC = (1, 0, 1)


def _pad(c):
    return (c + cmnn.CALIGN - 1) // cmnn.CALIGN * cmnn.CALIGN


class UNet3D:
    def __init__(self, dims, in_ch=2, out_ch=3, widths=(32, 64, 96), seed=0, device="cuda:0"):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.dims = tuple(int(v) for v in dims)  # (d, h, w) at full resolution
        assert all(v % 4 == 0 for v in self.dims), "spatial extents must be multiples of 4"
        self.in_ch, self.out_ch = in_ch, out_ch
        self.cin0, self.cout_head = _pad(in_ch), _pad(out_ch)
        w0, w1, w2 = widths
        spec = [  # name, cin (padded), cout (padded), real cin, real cout, activation
            ("e0a", self.cin0, w0, in_ch, w0, cmnn.ACT_LEAKY), ("e0b", w0, w0, w0, w0, cmnn.ACT_LEAKY),
            ("e1a", w0, w1, w0, w1, cmnn.ACT_LEAKY), ("e1b", w1, w1, w1, w1, cmnn.ACT_LEAKY),
            ("ma", w1, w2, w1, w2, cmnn.ACT_LEAKY), ("mb", 2 * w2, w2, 2 * w2, w2, cmnn.ACT_LEAKY),
            ("d1a", w1 + w2, w1, w1 + w2, w1, cmnn.ACT_LEAKY), ("d1b", w1, w1, w1, w1, cmnn.ACT_LEAKY),
            ("d0a", w0 + w1, w0, w0 + w1, w0, cmnn.ACT_LEAKY), ("d0b", w0, w0, w0, w0, cmnn.ACT_LEAKY),
            ("head", w0, self.cout_head, w0, out_ch, cmnn.ACT_NONE),
        ]
        self.widths = widths
        self.layers = {}
        sizes = []
        for name, ci, co, rci, rco, act in spec:
            sizes.append(27 * co * ci + co)
        total = sum(sizes)
        f32 = dict(dtype=torch.float32, device=self.device)
        self.params = torch.zeros(total, **f32)
        self.grads = torch.zeros(total, **f32)
        self.m = torch.zeros(total, **f32)
        self.v = torch.zeros(total, **f32)
        g = np.random.Generator(np.random.PCG64(seed))
        init = np.zeros(total, np.float32)
        off = 0
        for (name, ci, co, rci, rco, act), n in zip(spec, sizes):
            w = np.zeros((27, co, ci), np.float32)
            # He initialisation over the real fan-in (27 taps x real input channels)
            w[:, :rco, :rci] = g.standard_normal((27, rco, rci)) * np.sqrt(2.0 / (27 * rci))
            init[off:off + 27 * co * ci] = w.ravel()
            L = dict(name=name, cin=ci, cout=co, act=act, off=off, nw=27 * co * ci)
            L["w"] = self.params[off:off + 27 * co * ci].view(27, co, ci)
            L["b"] = self.params[off + 27 * co * ci:off + n]
            L["dw"] = self.grads[off:off + 27 * co * ci].view(27, co, ci)
            L["db"] = self.grads[off + 27 * co * ci:off + n]
            L["wf"] = torch.empty((27, co, ci), dtype=torch.bfloat16, device=self.device)
            L["wt"] = torch.empty((27, ci, co), dtype=torch.bfloat16, device=self.device)
            self.layers[name] = L
            off += n
        self.params.copy_(torch.from_numpy(init))
        self.nparams = total
        self.nparams_real = sum(27 * rco * rci + rco for (_, _, _, rci, rco, _) in spec)
        self.step_count = 0
        self._ws = None
        self._mws = None
        self._cws = None
        self.grad_norm = None
        self._jobs = None
        self.pack()

    # -- parameters
    def pack(self):
        if self._jobs is None:  # the tensors never move, so the descriptors are built once
            self._jobs = cmnn.pack_jobs([(L["w"], L["cin"], L["cout"], L["wf"], L["wt"])
                                         for L in self.layers.values()])
        cmnn.pack_weights_batch(self._jobs)

    def state_dict(self):
        return {"params": self.params.detach().cpu().numpy().copy(), "widths": np.array(self.widths),
                "dims": np.array(self.dims), "in_ch": self.in_ch, "out_ch": self.out_ch}

    def load_state(self, params):
        self.params.copy_(self.torch.as_tensor(np.asarray(params, np.float32), device=self.device))
        self.pack()

    # -- geometry helpers
    def geoms(self, n):
        d, h, w = self.dims
        return [cmnn.geom(n, d >> k, h >> k, w >> k, PERIODIC) for k in range(3)]

    def _t(self, n, level, c):
        d, h, w = self.dims
        return self.torch.empty((n, d >> level, h >> level, w >> level, c), dtype=self.torch.bfloat16,
                                device=self.device)

    def _conv(self, name, g, x, level):
        L = self.layers[name]
        y = self._t(g.n, level, L["cout"])
        cmnn.conv_fwd(g, x, L["cin"], L["wf"], L["b"], L["cout"], L["act"], y)
        return y

    # -- forward
    def forward(self, x):
        """x: BF16 [n, d, h, w, cin0] -> BF16 [n, d, h, w, cout_head]; keeps
        the activations for backward()."""
        n = x.shape[0]
        g0, g1, g2 = self.geoms(n)
        w0, w1, w2 = self.widths
        A = {"x": x}
        A["e0a"] = self._conv("e0a", g0, x, 0)
        A["s0"] = self._conv("e0b", g0, A["e0a"], 0)
        A["p0"] = self._t(n, 1, w0)
        cmnn.pool2_fwd(g0, A["s0"], w0, A["p0"])
        A["e1a"] = self._conv("e1a", g1, A["p0"], 1)
        A["s1"] = self._conv("e1b", g1, A["e1a"], 1)
        A["p1"] = self._t(n, 2, w1)
        cmnn.pool2_fwd(g1, A["s1"], w1, A["p1"])
        A["ma"] = self._conv("ma", g2, A["p1"], 2)
        A["cm"] = self._t(n, 2, 2 * w2)
        cmnn.channel_mean_concat(g2, A["ma"], w2, A["cm"], self._mean_ws(g2, w2))
        A["mb"] = self._conv("mb", g2, A["cm"], 2)
        A["c1"] = self._t(n, 1, w1 + w2)
        cmnn.up2_concat_fwd(g2, A["s1"], w1, A["mb"], w2, A["c1"])
        A["d1a"] = self._conv("d1a", g1, A["c1"], 1)
        A["d1b"] = self._conv("d1b", g1, A["d1a"], 1)
        A["c0"] = self._t(n, 0, w0 + w1)
        cmnn.up2_concat_fwd(g1, A["s0"], w0, A["d1b"], w1, A["c0"])
        A["d0a"] = self._conv("d0a", g0, A["c0"], 0)
        A["d0b"] = self._conv("d0b", g0, A["d0a"], 0)
        A["y"] = self._conv("head", g0, A["d0b"], 0)
        self.acts = A
        return A["y"]

    # -- backward
    def _workspace(self, n):
        g0, g1, g2 = self.geoms(n)
        need = 0
        for name, L in self.layers.items():
            g = {"e0a": g0, "e0b": g0, "d0a": g0, "d0b": g0, "head": g0, "e1a": g1, "e1b": g1, "d1a": g1,
                 "d1b": g1, "ma": g2, "mb": g2}[name]
            need = max(need, cmnn.conv_bwd_weight_workspace(g, L["cin"], L["cout"]))
        if self._ws is None or self._ws.numel() * 4 < need:
            self._ws = self.torch.empty((need + 3) // 4, dtype=self.torch.float32, device=self.device)
        return self._ws

    def _mean_ws(self, g, c):
        need = cmnn.channel_mean_workspace(g, c)
        if self._mws is None or self._mws.numel() * 4 < need:
            self._mws = self.torch.empty((need + 3) // 4, dtype=self.torch.float32, device=self.device)
        return self._mws

    def _conv_bwd(self, name, g, x, y, dy, level, need_dx=True, pre=False, into=None):
        """dy: gradient w.r.t. the layer output y, or with pre=True already
        w.r.t. its pre-activation.  Returns the gradient w.r.t. x; with into =
        the name of the layer whose activation output x is, the data-gradient
        kernel applies that activation's gradient too and returns the gradient
        w.r.t. that layer's pre-activation."""
        L = self.layers[name]
        if L["act"] != cmnn.ACT_NONE and not pre:
            dpre = self.torch.empty_like(dy)
            cmnn.act_bwd(y, dy, dpre, L["act"])
        else:
            dpre = dy
        cmnn.conv_bwd_weight(g, x, L["cin"], dpre, L["cout"], L["dw"], L["db"], self._ws)
        if not need_dx:
            return None
        dx = self._t(g.n, level, L["cin"])
        if into is not None:
            cmnn.conv_bwd_data_act(g, dpre, L["cout"], L["wt"], L["cin"], x, self.layers[into]["act"], dx)
        else:
            cmnn.conv_bwd_data(g, dpre, L["cout"], L["wt"], L["cin"], dx)
        return dx

    def backward(self, dy):
        """dy: BF16 gradient of the loss w.r.t. the output; fills self.grads."""
        A = self.acts
        n = dy.shape[0]
        g0, g1, g2 = self.geoms(n)
        w0, w1, w2 = self.widths
        self._workspace(n)
        # where a layer's input is the activation output of the layer below
        # (not a concatenation, pooling or sum), its data gradient also applies
        # that activation's gradient ("into"), and the layer below takes it as
        # its pre-activation gradient (pre=True); the skip joins apply it too.
        # The concatenations' gradients dc0, dc1, dcm are read in place: the
        # upsampled part by up2_bwd_act, the skip part by pool2_bwd_add_act,
        # both parts of dcm by channel_mean_add_act.
        act = {k: L["act"] for k, L in self.layers.items()}
        d = self._conv_bwd("head", g0, A["d0b"], A["y"], dy, 0, into="d0b")
        d = self._conv_bwd("d0b", g0, A["d0a"], A["d0b"], d, 0, pre=True, into="d0a")
        dc0 = self._conv_bwd("d0a", g0, A["c0"], A["d0a"], d, 0, pre=True)
        d = self._t(n, 1, w1)
        cmnn.up2_bwd_act(g1, dc0, w0, w0 + w1, w1, A["d1b"], act["d1b"], d)
        d = self._conv_bwd("d1b", g1, A["d1a"], A["d1b"], d, 1, pre=True, into="d1a")
        dc1 = self._conv_bwd("d1a", g1, A["c1"], A["d1a"], d, 1, pre=True)
        d = self._t(n, 2, w2)
        cmnn.up2_bwd_act(g2, dc1, w1, w1 + w2, w2, A["mb"], act["mb"], d)
        dcm = self._conv_bwd("mb", g2, A["cm"], A["mb"], d, 2, pre=True)
        d = self._t(n, 2, w2)
        # the mean map is self-adjoint: ma's gradient is the first part of dcm
        # plus the broadcast channel means of the second
        cmnn.channel_mean_add_act(g2, dcm, w2, 2 * w2, w2, dcm, 0, 2 * w2, A["ma"], act["ma"], d,
                                  self._mean_ws(g2, w2))
        d = self._conv_bwd("ma", g2, A["p1"], A["ma"], d, 2, pre=True)
        ds1 = self._t(n, 1, w1)
        cmnn.pool2_bwd_add_act(g1, d, w1, dc1, 0, w1 + w2, A["s1"], act["e1b"], ds1)
        d = self._conv_bwd("e1b", g1, A["e1a"], A["s1"], ds1, 1, pre=True, into="e1a")
        d = self._conv_bwd("e1a", g1, A["p0"], A["e1a"], d, 1, pre=True)
        ds0 = self._t(n, 0, w0)
        cmnn.pool2_bwd_add_act(g0, d, w0, dc0, 0, w0 + w1, A["s0"], act["e0b"], ds0)
        d = self._conv_bwd("e0b", g0, A["e0a"], A["s0"], ds0, 0, pre=True, into="e0a")
        self._conv_bwd("e0a", g0, A["x"], A["e0a"], d, 0, need_dx=False, pre=True)

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0, clip=None):
        """One Adam update from self.grads.  clip: global gradient-norm limit
        (0 measures only); the pre-clip norm and the applied scale land in
        self.grad_norm (device FP32[2])."""
        if clip is not None:
            if self._cws is None:
                self._cws = self.torch.empty(cmnn.clip_grad_norm_workspace(self.nparams) // 4,
                                             dtype=self.torch.float32, device=self.device)
                self.grad_norm = self.torch.zeros(2, dtype=self.torch.float32, device=self.device)
            cmnn.clip_grad_norm(self.grads, float(clip), self.grad_norm, self._cws)
        self.step_count += 1
        cmnn.adam(self.params, self.grads, self.m, self.v, lr, beta1, beta2, eps, weight_decay, self.step_count)
        self.pack()

    def flops_per_sample(self):
        """Multiply-add FLOPs (2 per MAC) of one forward pass per sample."""
        d, h, w = self.dims
        nv = [d * h * w >> (3 * k) for k in range(3)]
        lvl = {"e0a": 0, "e0b": 0, "d0a": 0, "d0b": 0, "head": 0, "e1a": 1, "e1b": 1, "d1a": 1, "d1b": 1, "ma": 2,
               "mb": 2}
        return sum(2 * 27 * L["cin"] * L["cout"] * nv[lvl[k]] for k, L in self.layers.items())
