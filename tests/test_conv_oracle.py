"""Pins of the FP64 network oracle (oracle/conv_oracle.py) against independent
definitions: FFT circular correlation, scipy's correlate on explicitly padded
arrays, delta kernels, central finite differences and adjoint identities."""
import numpy as np
import pytest
import scipy.signal

from oracle import conv_oracle as C
import workloads as W


def rnd(shape, seed):
    return W.generator(seed).standard_normal(shape)


def test_delta_and_shift_kernels():
    x = rnd((2, 4, 5, 6, 3), 1)
    w = np.zeros((27, 3, 3))
    w[13] = np.eye(3)  # centre tap
    np.testing.assert_array_equal(C.conv3d(x, w), x)
    w = np.zeros((27, 3, 3))
    w[14] = np.eye(3)  # tap (0, 0, +1): reads x at w + 1 (periodic)
    np.testing.assert_array_equal(C.conv3d(x, w, periodic=(1, 1, 1)), np.roll(x, -1, axis=3))


def test_periodic_conv_is_fft_circular_correlation():
    x = rnd((1, 6, 5, 8, 2), 2)
    w = rnd((27, 3, 2), 3)
    y = C.conv3d(x, w, periodic=(1, 1, 1))
    k = np.zeros((6, 5, 8, 3, 2))  # kernel embedded at its offsets
    for t, (dz, dy, dx) in enumerate(C.taps()):
        k[dz % 6, dy % 5, dx % 8] += w[t]
    X = np.fft.fftn(x[0], axes=(0, 1, 2))
    K = np.fft.fftn(k, axes=(0, 1, 2))
    # y[v, o] = sum_u x[v + u, i] k[u, o, i]  ->  Y = sum_i X_i * conj(K_oi) (real inputs)
    Y = np.einsum("dhwi,dhwoi->dhwo", X, np.conj(K))
    ref = np.real(np.fft.ifftn(Y, axes=(0, 1, 2)))
    np.testing.assert_allclose(y[0], ref, atol=1e-12)


def test_mixed_padding_matches_scipy_on_padded_input():
    x = rnd((1, 4, 5, 6, 2), 4)
    w = rnd((27, 2, 2), 5)
    b = rnd((2,), 6)
    y = C.conv3d(x, w, b, periodic=(1, 0, 1))
    xp = np.pad(x[0], ((1, 1), (0, 0), (1, 1), (0, 0)), mode="wrap")
    xp = np.pad(xp, ((0, 0), (1, 1), (0, 0), (0, 0)), mode="constant")
    ref = np.zeros_like(y[0])
    for o in range(2):
        for i in range(2):
            k = w[:, o, i].reshape(3, 3, 3)
            ref[..., o] += scipy.signal.correlate(xp[..., i], k, mode="valid")
        ref[..., o] += b[o]
    np.testing.assert_allclose(y[0], ref, atol=1e-12)


@pytest.mark.parametrize("periodic", [(1, 0, 1), (0, 1, 0)])
def test_conv_gradients_by_finite_differences(periodic):
    x = rnd((1, 3, 4, 5, 2), 7)
    w = rnd((27, 3, 2), 8)
    b = rnd((3,), 9)
    r = rnd((1, 3, 4, 5, 3), 10)
    loss = lambda x_, w_, b_: float((C.conv3d(x_, w_, b_, periodic) * r).sum())  # noqa: E731
    dx, dw, db = C.conv3d_grads(x, w, r, periodic)
    h = 1e-6
    g = W.generator(11)
    for _ in range(6):
        idx = tuple(int(g.integers(s)) for s in x.shape)
        e = np.zeros_like(x)
        e[idx] = h
        assert abs((loss(x + e, w, b) - loss(x - e, w, b)) / (2 * h) - dx[idx]) < 1e-6
        idx = tuple(int(g.integers(s)) for s in w.shape)
        e = np.zeros_like(w)
        e[idx] = h
        assert abs((loss(x, w + e, b) - loss(x, w - e, b)) / (2 * h) - dw[idx]) < 1e-6
    e = np.zeros(3)
    e[1] = h
    assert abs((loss(x, w, b + e) - loss(x, w, b - e)) / (2 * h) - db[1]) < 1e-6


def test_pool_and_upsample_adjoints():
    x = rnd((2, 4, 6, 8, 3), 12)
    y = rnd((2, 2, 3, 4, 3), 13)
    assert abs((C.pool2(x) * y).sum() - (x * C.pool2_grad(y)).sum()) < 1e-12
    assert abs((C.up2(y) * x).sum() - (y * C.up2_grad(x)).sum()) < 1e-12
    np.testing.assert_allclose(C.pool2(C.up2(y)), y, atol=1e-15)


def test_leaky_gradient_and_mse_finite_differences():
    y = rnd((50,), 14)
    dy = rnd((50,), 15)
    np.testing.assert_array_equal(C.leaky_grad_from_output(C.leaky(y), dy), np.where(y > 0, dy, C.LEAK * dy))
    pred = rnd((40, 4), 16)
    tgt = rnd((3, 40), 17)
    wt = (rnd((40,), 18) > 0).astype(float)
    loss, g = C.mse(pred, tgt, wt)
    h = 1e-6
    for idx in [(3, 0), (7, 2), (11, 1), (5, 3)]:
        e = np.zeros_like(pred)
        e[idx] = h
        num = (C.mse(pred + e, tgt, wt)[0] - C.mse(pred - e, tgt, wt)[0]) / (2 * h)
        assert abs(num - g[idx]) < 1e-8


def test_adam_first_step_is_sign_step():
    # with zero moments, the first bias-corrected Adam step is lr * g / (|g| + eps)
    p = rnd((10,), 19)
    g = rnd((10,), 20)
    p1, _, _ = C.adam(p, g, np.zeros(10), np.zeros(10), 1e-2, 0.9, 0.999, 1e-12, 0.0, 1)
    np.testing.assert_allclose(p1, p - 1e-2 * np.sign(g), atol=1e-9)


def test_channel_mean_is_symmetric_projection():
    x = rnd((2, 3, 4, 5, 3), 21)
    y = rnd((2, 3, 4, 5, 3), 22)
    P = C.channel_mean
    np.testing.assert_allclose(P(P(x)), P(x), atol=1e-15)
    assert abs((P(x) * y).sum() - (x * P(y)).sum()) < 1e-12
    np.testing.assert_allclose(P(x)[1, 2, 3, 4], x[1].reshape(-1, 3).mean(axis=0), atol=1e-15)


def test_clip_grad_norm_projects_onto_ball():
    g = rnd((7, 5), 23)
    n = np.linalg.norm(g)
    c, n0 = C.clip_grad_norm(g, 0.5 * n)
    assert n0 == pytest.approx(n)
    assert np.linalg.norm(c) == pytest.approx(0.5 * n)
    np.testing.assert_allclose(c / np.linalg.norm(c), g / n, atol=1e-15)  # direction kept
    np.testing.assert_array_equal(C.clip_grad_norm(g, 2 * n)[0], g)  # inside the ball: unchanged
    np.testing.assert_array_equal(C.clip_grad_norm(g, 0.0)[0], g)  # 0: measure only
