"""Pins of the reference network: the strided convolution against scipy's correlation, GELU
against the normal distribution function, pooling and the embedding at closed-form points, and
the hand-derived gradient against central finite differences (FP64)."""
import math

import numpy as np
import pytest
from scipy import signal, stats

from oracle import cnn


def test_conv_matches_scipy_correlation_subsampled():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 8, 8))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    out = cnn.conv_s2(x, W, b)
    for co in range(4):
        full = sum(signal.correlate2d(np.pad(x[ci], 1), W[co, ci], mode="valid")
                   for ci in range(3))
        assert np.allclose(out[co], full[::2, ::2] + b[co], rtol=1e-13, atol=1e-13)


def test_conv_backward_is_the_adjoint():
    """<conv(x) - b, y> = <x, conv_backward_x(y)>: the data gradient is the transposed map."""
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 8, 8))
    W = rng.standard_normal((3, 2, 3, 3))
    y = rng.standard_normal((3, 4, 4))
    lhs = np.sum((cnn.conv_s2(x, W, np.zeros(3))) * y)
    dx, dW, db = cnn.conv_s2_backward(x, W, y)
    assert abs(lhs - np.sum(x * dx)) <= 1e-12 * abs(lhs)
    assert abs(lhs - np.sum(W * dW)) <= 1e-12 * abs(lhs)
    assert np.allclose(db, y.sum(axis=(1, 2)))


def test_gelu_and_derivative():
    z = np.linspace(-5, 5, 101)
    assert np.allclose(cnn.gelu(z), z * stats.norm.cdf(z), rtol=1e-14, atol=1e-15)
    h = 1e-6
    fd = (cnn.gelu(z + h) - cnn.gelu(z - h)) / (2 * h)
    assert np.allclose(cnn.gelu_grad(z), fd, rtol=1e-8, atol=1e-9)


def test_pool_and_embedding_closed_forms():
    img = np.arange(64 * 64, dtype=np.float64).reshape(64, 64)
    p = cnn.pool2(img)
    assert p.shape == (32, 32)
    # mean of rows 2i, 2i+1 and columns 2j, 2j+1 of i*64 + j
    i, j = np.meshgrid(np.arange(32), np.arange(32), indexing="ij")
    assert np.array_equal(p, 128 * i + 2 * j + 32.5)
    e0 = cnn.embed(0)
    assert np.array_equal(e0[0::2], np.zeros(16)) and np.array_equal(e0[1::2], np.ones(16))
    e = cnn.embed(7)
    assert e[0] == math.sin(7) and e[1] == math.cos(7)
    assert abs(e[30] - math.sin(7 * 10000.0 ** (-15 / 16))) <= 1e-16


def test_param_count():
    k = 40
    assert cnn.param_count(k) == 16 * 9 + 16 + 32 * 144 + 32 + 64 * 288 + 64 + k * 96 + k


@pytest.fixture(scope="module")
def small_problem():
    rng = np.random.default_rng(2)
    k = 6
    theta = cnn.init_params(k, rng)
    theta[cnn.param_count(k) - k:] = rng.standard_normal(k) * 0.1     # nonzero head bias
    for l in range(3):                                                 # nonzero conv biases
        o = sum(int(np.prod(s)) for s in cnn.shapes(k)[:2 * l + 1])
        theta[o:o + cnn.CH[l + 1]] = rng.standard_normal(cnn.CH[l + 1]) * 0.1
    imgs = rng.uniform(0, 1, (2, 64, 64))
    steps = np.array([3, 58])
    target = rng.standard_normal((2, k))
    return k, theta, imgs, steps, target


def test_gradient_matches_central_differences(small_problem):
    k, theta, imgs, steps, target = small_problem
    L, g = cnn.loss_and_grad(theta, k, imgs, steps, target)
    a = cnn.forward(theta, k, imgs, steps)
    assert abs(L - np.mean((a - target) ** 2)) <= 1e-14 * L
    rng = np.random.default_rng(3)
    sizes = [int(np.prod(s)) for s in cnn.shapes(k)]
    offs = np.cumsum([0] + sizes)
    # every bias, and a sample of each weight tensor
    idx = []
    for t in range(len(sizes)):
        if t % 2 == 1 or sizes[t] <= 16:
            idx += list(range(offs[t], offs[t + 1]))
        else:
            idx += list(rng.choice(np.arange(offs[t], offs[t + 1]), 12, replace=False))
    h = 1e-5
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        Lp = np.mean((cnn.forward(tp, k, imgs, steps) - target) ** 2)
        Lm = np.mean((cnn.forward(tm, k, imgs, steps) - target) ** 2)
        fd = (Lp - Lm) / (2 * h)
        assert abs(g[i] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), i


def test_composition_on_a_hand_computable_network():
    """Centre-tap identity kernels on channel 0 make each layer keep every second position of
    channel 0 and apply GELU; the head reads feature 0 and the embedding's cos(n): alpha_0 is the
    mean of GELU(GELU(GELU(pooled[8y][8x]))), alpha_1 = cos(n)."""
    k = 2
    theta = np.zeros(cnn.param_count(k))
    W1, b1, W2, b2, W3, b3, Wl, bl = cnn.unpack(theta, k)    # views into theta
    for W in (W1, W2, W3):
        W[0, 0, 1, 1] = 1.0
    Wl[0, 0] = 1.0
    Wl[1, cnn.CH[3] + 1] = 1.0
    bl[1] = 0.25
    rng = np.random.default_rng(4)
    img = rng.uniform(-1, 2, (64, 64))
    pooled = img.reshape(32, 2, 32, 2).mean(axis=(1, 3))
    g = lambda z: z * stats.norm.cdf(z)                      # noqa: E731
    expect0 = np.mean(g(g(g(pooled[::8, ::8]))))
    alpha = cnn.forward_one(theta, k, img, 11)
    assert abs(alpha[0] - expect0) <= 1e-14
    assert abs(alpha[1] - (math.cos(11) + 0.25)) <= 1e-15
