"""FP64 CPU oracle of the warm-start network operations (TEST INFRASTRUCTURE
ONLY: used by tests/ and never by the product package; shares no code with the
HIP kernels of libcmnn).

Definitions written out with numpy in float64 on NDHWC arrays [n, d, h, w, c]:
- 3x3x3 "same" cross-correlation with per-axis periodic or zero padding,
  y[v, co] = sum_t sum_ci x[v + off(t), ci] w[t, co, ci] + b[co], tap
  t = (dz+1)*9 + (dy+1)*3 + (dx+1);
- its gradients, obtained as the adjoint of each shifted read (a zero-padded
  read at v + off is adjoint to a zero-padded write at v - off);
- leaky ReLU (slope 0.1), 2x2x2 average pooling, 2x nearest upsampling,
  channel concatenation, per-sample channel means, masked mean-squared
  error, gradient-norm clipping, Adam.
"""
import numpy as np

LEAK = 0.1


def taps():
    return [(t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1) for t in range(27)]


def shifted(x, off, periodic):
    """out[v] = x[v + off] along (d, h, w), periodic or zero-padded per axis."""
    out = x
    for axis, (o, per) in enumerate(zip(off, periodic)):
        ax = axis + 1
        if o == 0:
            continue
        if per:
            out = np.roll(out, -o, axis=ax)
        else:
            n = out.shape[ax]
            res = np.zeros_like(out)
            src = [slice(None)] * out.ndim
            dst = [slice(None)] * out.ndim
            if o > 0:
                src[ax] = slice(o, n)
                dst[ax] = slice(0, n - o)
            else:
                src[ax] = slice(0, n + o)
                dst[ax] = slice(-o, n)
            res[tuple(dst)] = out[tuple(src)]
            out = res
    return out


def conv3d(x, w, b=None, periodic=(1, 0, 1)):
    """x [n,d,h,w,cin], w [27,cout,cin], b [cout] -> y [n,d,h,w,cout]."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    y = np.zeros(x.shape[:4] + (w.shape[1],))
    for t, off in enumerate(taps()):
        y += shifted(x, off, periodic) @ w[t].T
    if b is not None:
        y += np.asarray(b, np.float64)
    return y


def conv3d_grads(x, w, dy, periodic=(1, 0, 1)):
    """Gradients of sum(dy * conv3d(x, w, b)) with respect to x, w and b."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    dy = np.asarray(dy, np.float64)
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for t, off in enumerate(taps()):
        xs = shifted(x, off, periodic)
        dw[t] = np.einsum("ndhwo,ndhwi->oi", dy, xs)
        # adjoint of the read x[v + off]: a write of dy @ w[t] at v + off
        dx += shifted(dy @ w[t], tuple(-o for o in off), periodic)
    db = dy.sum(axis=(0, 1, 2, 3))
    return dx, dw, db


def leaky(x):
    return np.where(x > 0, x, LEAK * x)


def leaky_grad_from_output(y, dy):
    return np.where(y > 0, dy, LEAK * dy)


def pool2(x):
    n, d, h, w, c = x.shape
    return x.reshape(n, d // 2, 2, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4, 6))


def pool2_grad(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def up2(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def up2_grad(dy):
    n, d, h, w, c = dy.shape
    return dy.reshape(n, d // 2, 2, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4, 6))


def channel_mean(x):
    """Per-sample channel means broadcast back over the voxels (a symmetric projection)."""
    return np.broadcast_to(x.mean(axis=(1, 2, 3), keepdims=True), x.shape).copy()


def mse(pred, target, weight):
    """pred [nvox, c] (first creal channels used), target [creal, nvox],
    weight [nvox] -> (loss, dpred)."""
    creal = target.shape[0]
    d = pred[:, :creal] - target.T
    norm = creal * weight.sum()
    loss = float((weight[:, None] * d * d).sum() / norm)
    g = np.zeros_like(pred, dtype=np.float64)
    g[:, :creal] = 2.0 * weight[:, None] * d / norm
    return loss, g


def clip_grad_norm(g, max_norm):
    """(g * min(1, max_norm / ||g||), ||g||); max_norm = 0 leaves g unchanged."""
    norm = float(np.sqrt((np.asarray(g, np.float64) ** 2).sum()))
    scale = max_norm / norm if 0 < max_norm < norm else 1.0
    return g * scale, norm


def adam(p, g, m, v, lr, b1, b2, eps, wd, step):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    p = p - lr * (mh / (np.sqrt(vh) + eps) + wd * p)
    return p, m, v
