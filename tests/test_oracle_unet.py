"""Pins of the network oracle (oracle/unet.py): its convolution against scipy's
N-d correlation, its backward pass against central finite differences in FP64,
adjointness of the resampling operators, the residual identity, and the first Adam
step's closed form."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import unet

RNG = np.random.default_rng(3141)


def test_conv_is_scipy_correlation_with_zero_padding():
    x = RNG.standard_normal((3, 6, 5, 7))
    w = RNG.standard_normal((2, 3, 3, 3, 3))
    b = RNG.standard_normal(2)
    out = unet.conv3d(x, w, b)
    for o in range(2):
        want = b[o] + sum(ndimage.correlate(x[c], w[o, c], mode="constant", cval=0.0) for c in range(3))
        np.testing.assert_allclose(out[o], want, rtol=1e-12, atol=1e-12)


def _fd(f, x, idx, h=1e-6):
    xp = x.copy()
    xm = x.copy()
    xp.flat[idx] += h
    xm.flat[idx] -= h
    return (f(xp) - f(xm)) / (2 * h)


def test_conv_backward_matches_finite_differences():
    x = RNG.standard_normal((2, 4, 5, 3))
    w = RNG.standard_normal((3, 2, 3, 3, 3))
    b = RNG.standard_normal(3)
    g = RNG.standard_normal((3, 4, 5, 3))
    gx, gw, gb = unet.conv3d_backward(x, w, g)
    loss_x = lambda xx: float(np.sum(g * unet.conv3d(xx, w, b)))
    loss_w = lambda ww: float(np.sum(g * unet.conv3d(x, ww, b)))
    loss_b = lambda bb: float(np.sum(g * unet.conv3d(x, w, bb)))
    for idx in RNG.choice(x.size, 12, replace=False):
        assert abs(gx.flat[idx] - _fd(loss_x, x, idx)) < 1e-6 * (1 + abs(gx.flat[idx]))
    for idx in RNG.choice(w.size, 12, replace=False):
        assert abs(gw.flat[idx] - _fd(loss_w, w, idx)) < 1e-6 * (1 + abs(gw.flat[idx]))
    for idx in range(3):
        assert abs(gb[idx] - _fd(loss_b, b, idx)) < 1e-6 * (1 + abs(gb[idx]))


def test_resampling_operators_are_adjoint():
    a = RNG.standard_normal((2, 3, 3, 3))
    c = RNG.standard_normal((2, 6, 6, 6))
    assert np.isclose(np.sum(unet.up2(a) * c), np.sum(a * unet.up2_backward(c)))
    assert np.isclose(np.sum(unet.pool2(c) * a), np.sum(c * unet.pool2_backward(a)))
    assert np.allclose(unet.pool2(unet.up2(a)), a)


def _theta(scale=0.3, seed=7):
    rng = np.random.default_rng(seed)
    th = []
    for _, ci, co, k in unet.LAYERS:
        th.append(rng.standard_normal(co * ci * k ** 3) * scale / np.sqrt(ci * k ** 3))
        th.append(rng.standard_normal(co) * 0.1)
    return np.concatenate(th)


def test_network_gradient_matches_finite_differences():
    theta = _theta()
    x = RNG.standard_normal((4, 4, 4))
    t = RNG.standard_normal((4, 4, 4))

    def loss_theta(th):
        return unet.mse(unet.forward(th, x)[0], t)[0]

    y, cache = unet.forward(theta, x)
    _, gy = unet.mse(y, t)
    gth, gx = unet.backward(theta, cache, gy)
    assert gth.size == theta.size == unet.param_count()
    offs = np.cumsum([0] + [co * ci * k ** 3 + co for _, ci, co, k in unet.LAYERS])
    # a few parameters of every layer, weights and biases
    picks = []
    for i in range(len(unet.LAYERS)):
        picks += list(RNG.integers(offs[i], offs[i + 1], size=4)) + [offs[i + 1] - 1]
    for idx in picks:
        fd = _fd(loss_theta, theta, idx)
        assert abs(gth[idx] - fd) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (idx, gth[idx], fd)
    loss_x = lambda xx: unet.mse(unet.forward(theta, xx)[0], t)[0]
    for idx in RNG.choice(x.size, 6, replace=False):
        fd = _fd(loss_x, x, idx)
        assert abs(gx.flat[idx] - fd) <= 1e-6 * max(1.0, abs(fd)) + 1e-9


def test_zero_output_layer_is_the_identity():
    theta = _theta()
    p = unet.unpack(theta)
    p["out"][0][...] = 0.0
    p["out"][1][...] = 0.0
    x = RNG.standard_normal((8, 8, 8))
    y, _ = unet.forward(theta, x)
    assert np.array_equal(y, x)


def test_first_adam_step_moves_by_lr_times_sign():
    g = RNG.standard_normal(50)
    th = RNG.standard_normal(50)
    new, m, v = unet.adam_step(th, g, np.zeros(50), np.zeros(50), 1, lr=1e-3, eps=0.0)
    np.testing.assert_allclose(th - new, 1e-3 * np.sign(g), rtol=1e-12)


def test_bf16_rounding_is_nearest_with_ties_to_even():
    one = 1.0
    cases = {one + 2.0 ** -8: 1.0, one + 3 * 2.0 ** -8: one + 2.0 ** -6, one + 2.0 ** -7: one + 2.0 ** -7,
             -(one + 2.0 ** -8 + 2.0 ** -12): -(one + 2.0 ** -7), 3.0: 3.0}
    for a, want in cases.items():
        assert unet.bf16_round(np.array([a], np.float32))[0] == want, a
    # random values: the result has 8 significant bits and no 8-bit value is closer
    a = (RNG.standard_normal(2000) * 10.0 ** RNG.integers(-6, 6, 2000)).astype(np.float32)
    r = unet.bf16_round(a)
    e = np.floor(np.log2(np.abs(a.astype(np.float64))))
    ulp = 2.0 ** (e - 7)
    assert np.all(np.abs(r / ulp - np.round(r / ulp)) < 1e-9)             # on the 8-bit grid (or the next binade)
    assert np.all(np.abs(r - a) <= 0.5 * ulp * (1 + 1e-12))
