"""Float64 oracle of the learned distance correction (test infrastructure).

Not part of the paper: the paper's distance comes from the GP alone (Sec. III
and IV).  This is the residual network that the correction extension adds on
top of the GP distance: standardised features
    [d, log v, o, grad d (3), log(1 + n_local)]
feed three dense layers of width 64 with GELU (erf form, Hendrycks and Gimpel
2016) and a linear output r; the corrected distance is d + r where the GP
variance is at most ``gate`` and d elsewhere.  Training minimises the mean
squared error of d + r against the brute-force nearest-point distance with
Adam (Kingma and Ba 2015).

Flat parameter layout (8,897 numbers), shared with the C ABI:
    W1 [64 x 7], b1 [64], W2 [64 x 64], b2 [64], W3 [64 x 64], b3 [64],
    W4 [1 x 64], b4 [1]      (row-major, W[out, in])
Only the tests and the benchmark's CPU baseline use this module.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SHAPES = [(64, 7), (64,), (64, 64), (64,), (64, 64), (64,), (1, 64), (1,)]
NPARAM = sum(int(np.prod(s)) for s in SHAPES)
NFEAT = 7


def unflatten(flat):
    flat = np.asarray(flat, np.float64)
    assert flat.size == NPARAM
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(flat[o:o + n].reshape(s))
        o += n
    return out


def flatten(params):
    return np.concatenate([np.asarray(p, np.float64).ravel() for p in params])


def features(dist, var, occ, grad, n_local):
    """Raw (unstandardised) feature matrix [N, 7] from GP outputs."""
    return np.concatenate([
        np.asarray(dist, np.float64)[:, None],
        np.log(np.asarray(var, np.float64))[:, None],
        np.asarray(occ, np.float64)[:, None],
        np.asarray(grad, np.float64).reshape(-1, 3),
        np.log1p(np.asarray(n_local, np.float64))[:, None],
    ], axis=1)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(flat, z):
    """z: standardised features [N, 7] -> residual r [N] (and the cache)."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unflatten(flat)
    a0 = np.asarray(z, np.float64)
    p1 = a0 @ W1.T + b1
    a1 = gelu(p1)
    p2 = a1 @ W2.T + b2
    a2 = gelu(p2)
    p3 = a2 @ W3.T + b3
    a3 = gelu(p3)
    r = (a3 @ W4.T + b4)[:, 0]
    return r, (a0, p1, a1, p2, a2, p3, a3)


def loss_and_grad(flat, z, target):
    """Mean squared error of r against ``target`` (= truth - d) and its
    gradient with respect to the flat parameters (reverse mode)."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unflatten(flat)
    r, (a0, p1, a1, p2, a2, p3, a3) = forward(flat, z)
    n = r.shape[0]
    e = r - np.asarray(target, np.float64)
    loss = float(np.mean(e * e))
    g_r = (2.0 / n) * e[:, None]                 # dL/dr  [N, 1]
    gW4 = g_r.T @ a3
    gb4 = g_r.sum(0)
    g_a3 = g_r @ W4
    g_p3 = g_a3 * gelu_grad(p3)
    gW3 = g_p3.T @ a2
    gb3 = g_p3.sum(0)
    g_a2 = g_p3 @ W3
    g_p2 = g_a2 * gelu_grad(p2)
    gW2 = g_p2.T @ a1
    gb2 = g_p2.sum(0)
    g_a1 = g_p2 @ W2
    g_p1 = g_a1 * gelu_grad(p1)
    gW1 = g_p1.T @ a0
    gb1 = g_p1.sum(0)
    return loss, flatten([gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4])


class Adam:
    """Adam with bias correction, beta = (0.9, 0.999), eps = 1e-8."""

    def __init__(self, n, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, flat, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return flat - self.lr * mh / (np.sqrt(vh) + self.eps)


def corrected(dist, var, r, gate):
    """d + r where the GP variance is at most ``gate``, d elsewhere."""
    dist = np.asarray(dist, np.float64)
    return np.where(np.asarray(var) <= gate, dist + r, dist)
