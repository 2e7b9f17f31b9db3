"""Pins of the float64 MLP oracle: finite differences, GELU and Adam."""
import math

import numpy as np
from scipy.special import erf

from oracle import mlp as M


def _rand_params(seed):
    rng = np.random.default_rng(seed)
    flat = []
    for s in M.SHAPES:
        fan_in = s[1] if len(s) == 2 else 64
        flat.append(rng.normal(0, 1 / math.sqrt(fan_in), size=s))
    return M.flatten(flat)


def test_parameter_count():
    assert M.NPARAM == 8897


def test_backward_against_central_differences():
    rng = np.random.default_rng(0)
    flat = _rand_params(1)
    z = rng.normal(size=(32, 7))
    y = rng.normal(size=32) * 0.1
    _, g = M.loss_and_grad(flat, z, y)
    idx = rng.choice(M.NPARAM, 300, replace=False)
    h = 1e-6
    for i in idx:
        fp = flat.copy(); fp[i] += h
        fm = flat.copy(); fm[i] -= h
        lp, _ = M.loss_and_grad(fp, z, y)
        lm, _ = M.loss_and_grad(fm, z, y)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, i


def test_gelu_closed_form_points():
    # GELU(x) = x Phi(x): Phi(0) = 1/2, Phi(1) from erf(1/sqrt 2)
    assert M.gelu(np.array(0.0)) == 0.0
    assert abs(M.gelu(np.array(1.0)) - 0.5 * (1 + erf(1 / math.sqrt(2)))) < 1e-16
    x = np.linspace(-4, 4, 81)
    h = 1e-6
    fd = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    assert np.abs(fd - M.gelu_grad(x)).max() < 1e-8


def test_adam_first_step_moves_by_lr_times_sign():
    # with bias correction the first Adam step is lr * g / (|g| + eps)
    opt = M.Adam(4, lr=0.01)
    w = np.zeros(4)
    g = np.array([3.0, -2.0, 1e-3, 0.0])
    w1 = opt.step(w, g)
    assert np.allclose(w1, -0.01 * g / (np.abs(g) + 1e-8), atol=1e-15)


def test_training_reduces_loss_on_a_smooth_target():
    rng = np.random.default_rng(2)
    z = rng.normal(size=(512, 7))
    y = 0.1 * np.tanh(z[:, 0]) - 0.05 * z[:, 2] ** 2
    flat = _rand_params(3) * 0.5
    opt = M.Adam(M.NPARAM, lr=3e-3)
    l0, _ = M.loss_and_grad(flat, z, y)
    for _ in range(300):
        _, g = M.loss_and_grad(flat, z, y)
        flat = opt.step(flat, g)
    l1, _ = M.loss_and_grad(flat, z, y)
    assert l1 < 0.1 * l0


def test_gate():
    d = np.array([1.0, 2.0, 3.0])
    r = np.array([0.1, 0.2, 0.3])
    out = M.corrected(d, np.array([0.01, 0.05, 0.06]), r, gate=0.05)
    assert out.tolist() == [1.1, 2.2, 3.0]


def test_features_hand_built_row():
    # [d, log v, o, grad d (3), log(1 + n_local)], worked by hand:
    # log 0.02 = log 2 - log 100 = 0.693147... - 4.605170... = -3.912023...
    # log 38 = 3.637586...
    f = M.features([0.3], [0.02], [0.4], [[0.1, -0.2, 0.9]], [37])
    want = [0.3, -3.912023005428146, 0.4, 0.1, -0.2, 0.9, 3.6375861597263857]
    assert f.shape == (1, 7)
    assert np.abs(f[0] - want).max() < 1e-15
    # columns follow their inputs: permuting one input permutes one column
    g = M.features([1.0, 2.0], [1.0, math.e], [0.5, 0.25], [[1, 2, 3], [4, 5, 6]], [0, math.e - 1])
    assert g[:, 0].tolist() == [1.0, 2.0] and g[:, 2].tolist() == [0.5, 0.25]
    assert np.abs(g[:, 1] - [0.0, 1.0]).max() < 1e-15
    assert g[:, 3:6].tolist() == [[1, 2, 3], [4, 5, 6]]
    assert np.abs(g[:, 6] - [0.0, 1.0]).max() < 1e-15
