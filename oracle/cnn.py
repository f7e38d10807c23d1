"""Reference network of the learned starting guess, FP64 numpy (test infrastructure only).

The network maps a target's initial image (64 x 64, pooled 2 x 2 to 32 x 32) and the timestep
index n to k coefficients in the seed subspace (alpha_L, x0_L = V alpha_L):
  conv 3x3 stride 2 pad 1, 1 -> 16 channels (32 -> 16), GELU
  conv 3x3 stride 2 pad 1, 16 -> 32 (16 -> 8), GELU
  conv 3x3 stride 2 pad 1, 32 -> 64 (8 -> 4), GELU
  mean over the 4 x 4 positions -> 64 features, concatenated with a 32-wide sinusoidal
  embedding of n -> 96, linear -> k.
Loss: mean squared error over the batch and the k outputs.

Parameters are one flat vector in the order conv1.W (16, 1, 3, 3), conv1.b, conv2.W (32, 16, 3, 3),
conv2.b, conv3.W (64, 32, 3, 3), conv3.b, lin.W (k, 96), lin.b (k).  Images are (64, 64) arrays
indexed [i][j] with the unknown ordering p = i*64 + j.  Everything here is written plainly
(explicit convolution sums, hand-derived backward pass); the tests pin it against library
routines and central finite differences.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

CH = (1, 16, 32, 64)
EMB = 32
FEAT = CH[-1] + EMB


def shapes(k):
    out = []
    for l in range(3):
        out += [(CH[l + 1], CH[l], 3, 3), (CH[l + 1],)]
    out += [(k, FEAT), (k,)]
    return out


def param_count(k):
    return sum(int(np.prod(s)) for s in shapes(k))


def unpack(theta, k):
    parts, o = [], 0
    for s in shapes(k):
        c = int(np.prod(s))
        parts.append(theta[o:o + c].reshape(s))
        o += c
    return parts


def init_params(k, rng):
    """He-style normal initialisation of the weights, zero biases."""
    parts = []
    for s in shapes(k):
        if len(s) == 1:
            parts.append(np.zeros(s))
        else:
            fan_in = int(np.prod(s[1:]))
            parts.append(rng.standard_normal(s) * math.sqrt(2.0 / fan_in))
    return np.concatenate([p.reshape(-1) for p in parts])


def pool2(img):
    """2 x 2 average pooling of an (S, S) image."""
    S = img.shape[0] // 2
    return img.reshape(S, 2, S, 2).mean(axis=(1, 3))


def embed(n):
    """e[2i] = sin(n w_i), e[2i+1] = cos(n w_i), w_i = 10000^(-i/16), i < 16."""
    e = np.empty(EMB)
    for i in range(EMB // 2):
        w = 10000.0 ** (-i / (EMB // 2))
        e[2 * i] = math.sin(n * w)
        e[2 * i + 1] = math.cos(n * w)
    return e


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    cdf = 0.5 * (1.0 + erf(z / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return cdf + z * pdf


def conv_s2(x, W, b):
    """out[co, oy, ox] = b[co] + sum_{ci, ky, kx} W[co, ci, ky, kx] x[ci, 2oy+ky-1, 2ox+kx-1],
    zero outside x."""
    CI, S, _ = x.shape
    CO = W.shape[0]
    So = S // 2
    xp = np.zeros((CI, S + 2, S + 2))
    xp[:, 1:S + 1, 1:S + 1] = x
    out = np.empty((CO, So, So))
    for co in range(CO):
        acc = np.full((So, So), b[co])
        for ky in range(3):
            for kx in range(3):
                # sum over the input channels of W[co, ci, ky, kx] x[ci, 2oy+ky-1, 2ox+kx-1]
                win = xp[:, ky:ky + 2 * So:2, kx:kx + 2 * So:2]
                acc += np.tensordot(W[co, :, ky, kx], win, axes=1)
        out[co] = acc
    return out


def conv_s2_backward(x, W, dout):
    """Gradients of conv_s2 with respect to x, W and b, given d(loss)/d(out)."""
    CI, S, _ = x.shape
    CO, So = W.shape[0], dout.shape[1]
    xp = np.zeros((CI, S + 2, S + 2))
    xp[:, 1:S + 1, 1:S + 1] = x
    dW = np.zeros_like(W)
    dxp = np.zeros_like(xp)
    for co in range(CO):
        for ky in range(3):
            for kx in range(3):
                win = xp[:, ky:ky + 2 * So:2, kx:kx + 2 * So:2]          # (CI, So, So)
                dW[co, :, ky, kx] = np.sum(dout[co] * win, axis=(1, 2))
                dxp[:, ky:ky + 2 * So:2, kx:kx + 2 * So:2] += W[co, :, ky, kx][:, None, None] * dout[co]
    db = dout.sum(axis=(1, 2))
    return dxp[:, 1:S + 1, 1:S + 1], dW, db


def forward_one(theta, k, img64, n, keep=False):
    W1, b1, W2, b2, W3, b3, Wl, bl = unpack(theta, k)
    a = [pool2(np.asarray(img64, dtype=np.float64).reshape(64, 64))[None]]
    z = []
    for W, b in ((W1, b1), (W2, b2), (W3, b3)):
        z.append(conv_s2(a[-1], W, b))
        a.append(gelu(z[-1]))
    u = np.concatenate([a[-1].mean(axis=(1, 2)), embed(n)])
    alpha = Wl @ u + bl
    if keep:
        return alpha, (a, z, u)
    return alpha


def forward(theta, k, imgs, steps):
    return np.stack([forward_one(theta, k, im, n) for im, n in zip(imgs, steps)])


def loss_and_grad(theta, k, imgs, steps, target):
    """L = mean over batch and outputs of (alpha - target)^2, and dL/dtheta."""
    B = len(imgs)
    W1, b1, W2, b2, W3, b3, Wl, bl = unpack(theta, k)
    grads = [np.zeros(s) for s in shapes(k)]
    L = 0.0
    for bi in range(B):
        alpha, (a, z, u) = forward_one(theta, k, imgs[bi], steps[bi], keep=True)
        d = alpha - target[bi]
        L += np.sum(d * d)
        dalpha = 2.0 * d / (B * k)
        grads[6] += np.outer(dalpha, u)
        grads[7] += dalpha
        du = Wl.T @ dalpha
        S3 = a[3].shape[1]
        da = np.broadcast_to((du[:CH[3]] / (S3 * S3))[:, None, None], a[3].shape).copy()
        for l, (W, _) in reversed(list(enumerate(((W1, b1), (W2, b2), (W3, b3))))):
            dz = da * gelu_grad(z[l])
            dx, dW, db = conv_s2_backward(a[l], W, dz)
            grads[2 * l] += dW
            grads[2 * l + 1] += db
            da = dx
    return L / (B * k), np.concatenate([g.reshape(-1) for g in grads])
