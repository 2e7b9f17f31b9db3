"""GPU checks of the learned distance correction against the FP64 oracle
(oracle/mlp.py): the BF16 MFMA forward and backward, one Adam step, and the
held-out gain of a network trained on the GPU.

Tolerances (BF16 operands, FP32 accumulation):
  forward      |r - r_o| <= 1e-2 * (1 + |r_o|)
  gradient     per tensor cosine >= 0.999 and relative L2 <= 2e-2
  loss         relative 1e-2
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import mlp as OM
import paper_2407_09649_amd as P
from paper_2407_09649_amd import scenes as S

from parity import small_params

pytestmark = pytest.mark.gpu


def _ctx(dev, **kw):
    return P.Context(small_params(**kw), device=dev)


def _tensors(flat):
    return OM.unflatten(np.asarray(flat, np.float64))


def _z(feat, mean, std):
    return (np.asarray(feat, np.float64) - mean.astype(np.float64)) / std.astype(np.float64)


def test_forward_matches_oracle(dev):
    ctx = _ctx(dev)
    ctx.mlp_init(seed=7)
    mean = np.array([0.5, -3.0, 0.1, 0.0, 0.0, 0.0, 2.0], np.float32)
    std = np.array([0.7, 1.5, 0.2, 0.6, 0.6, 0.6, 1.1], np.float32)
    ctx.mlp_set_norm(mean, std)
    rng = np.random.default_rng(0)
    for n in (1, 31, 33, 1000):        # partial and whole 32-sample slices
        f = (mean + std * rng.normal(size=(n, 7))).astype(np.float32)
        r = ctx.mlp_forward(torch.from_numpy(f).to(dev)).cpu().numpy()
        ro, _ = OM.forward(ctx.mlp_get_weights(), _z(f, mean, std))
        assert np.all(np.abs(r - ro) <= 1e-2 * (1 + np.abs(ro))), (n, np.abs(r - ro).max())


@pytest.mark.parametrize("n", [32, 1000, 20000])
def test_gradient_matches_oracle(dev, n):
    ctx = _ctx(dev)
    ctx.mlp_init(seed=3)
    rng = np.random.default_rng(n)
    f = rng.normal(size=(n, 7)).astype(np.float32)
    t = (0.3 * rng.normal(size=n)).astype(np.float32)
    ctx.mlp_set_norm(np.zeros(7, np.float32), np.ones(7, np.float32))
    g, loss = ctx.mlp_grad(torch.from_numpy(f).to(dev), torch.from_numpy(t).to(dev))
    g = g.cpu().numpy().astype(np.float64)
    lo, go = OM.loss_and_grad(ctx.mlp_get_weights(), f.astype(np.float64), t.astype(np.float64))
    assert abs(loss / lo - 1) <= 1e-2
    for name, a, b in zip(("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"), _tensors(g), _tensors(go)):
        a, b = a.ravel(), b.ravel()
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300)
        rel = np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-300)
        assert cos >= 0.999 and rel <= 2e-2, (name, cos, rel)


def test_one_adam_step(dev):
    """A full-batch epoch is one Adam step; at t = 1 it moves every weight by
    lr g / (|g| + eps), so the oracle step from the oracle gradient must agree
    wherever the sign of g agrees."""
    ctx = _ctx(dev)
    ctx.mlp_init(seed=11)
    w0 = ctx.mlp_get_weights()
    rng = np.random.default_rng(5)
    n, lr = 4096, 1e-3
    f = rng.normal(size=(n, 7)).astype(np.float32)
    t = (0.3 * rng.normal(size=n)).astype(np.float32)
    ctx.mlp_train(torch.from_numpy(f).to(dev), torch.from_numpy(t).to(dev), epochs=1, batch=n, lr=lr, seed=1)
    w1 = ctx.mlp_get_weights().astype(np.float64)
    mean, std = ctx.mlp_get_norm()
    np.testing.assert_allclose(mean, f.astype(np.float64).mean(0), atol=1e-5)
    np.testing.assert_allclose(std, f.astype(np.float64).std(0), rtol=1e-5)
    _, go = OM.loss_and_grad(w0, _z(f, mean, std), t.astype(np.float64))
    adam = OM.Adam(OM.NPARAM, lr)
    wo = adam.step(w0.astype(np.float64), go)
    d = np.abs(w1 - wo)
    assert d.max() <= 2 * lr + 1e-6
    assert np.mean(d > 0.01 * lr) <= 0.05


def _pairs(ctx, dev, seed, nq):
    """(features, target = truth - d, d, truth, var, valid) of one sphere scene;
    the truth is the oracle's brute-force nearest-point distance."""
    sc = S.sphere_scene(seed, n_queries=0)
    q = S.sphere_eval_queries(seed + 50_000, nq)
    ctx.train(torch.from_numpy(sc.points).to(dev))
    qd = torch.from_numpy(q).to(dev)
    res = ctx.query(qd)
    feat = ctx.mlp_features(res)
    truth = O.nearest_distance(sc.points, q)
    d = res["dist"].cpu().numpy().astype(np.float64)
    v = res["valid"].cpu().numpy().astype(bool)
    var = res["var"].cpu().numpy()
    ok = v & np.isfinite(feat.cpu().numpy()).all(1)
    return feat, truth - d, d, truth, var, ok, qd


def test_trained_correction_gains_on_held_out_scene(dev):
    """Pairs the method generates (GP output vs brute-force truth) on four
    sphere scenes train the network on the GPU; on a fifth scene the corrected
    distance must have a lower error than the plain GP, and the gated query
    path must apply exactly d + r where the variance is at most the gate."""
    ctx = _ctx(dev, selection=P.SEL_KNN, knn_q=8, cluster_size=0.4)
    feats, tgts = [], []
    for seed in range(10000, 10004):
        f, t, _, _, _, ok, _ = _pairs(ctx, dev, seed, 25000)
        idx = torch.from_numpy(np.nonzero(ok)[0]).to(dev)
        feats.append(f[idx])
        tgts.append(torch.from_numpy(t[ok].astype(np.float32)).to(dev))
    feat = torch.cat(feats)
    tgt = torch.cat(tgts)
    ctx.mlp_init(seed=0)
    loss = ctx.mlp_train(feat, tgt, epochs=6, batch=512, lr=2e-3, seed=4)
    base = float((tgt.double() ** 2).mean())
    assert loss < 0.5 * base, (loss, base)
    # held-out scene
    f, t, d, truth, var, ok, qd = _pairs(ctx, dev, 20000, 25000)
    r = ctx.mlp_forward(f).cpu().numpy().astype(np.float64)
    e0 = np.mean((d[ok] - truth[ok]) ** 2)
    e1 = np.mean((d[ok] + r[ok] - truth[ok]) ** 2)
    assert e1 < 0.5 * e0, (e1, e0)
    # the fused, gated path of the query
    res = ctx.query(qd, correct=True)
    dc = res["dist"].cpu().numpy().astype(np.float64)
    gate = ctx.params.mlp_gate
    g = ok & (var <= gate)
    np.testing.assert_allclose(dc[g], d[g] + r[g], atol=1e-5)
    np.testing.assert_array_equal(dc[ok & ~g], d[ok & ~g])
    assert ctx.stats()["gated"] == int((res["valid"].cpu().numpy().astype(bool) & (var <= gate)).sum())


def test_features_match_oracle(dev):
    """gpdf_mlp_features on the outputs of a GP query, element by element
    against oracle.mlp.features on the same (FP32) outputs: the inputs pass
    through unchanged, the two logarithms within FP32 rounding."""
    sc = S.sphere_scene(10000)
    q = S.sphere_eval_queries(20000, 5000)
    with _ctx(dev, selection=P.SEL_KNN, knn_q=8) as ctx:
        ctx.train(torch.from_numpy(sc.points).to(dev))
        r = ctx.query(torch.from_numpy(q).to(dev))
        f = ctx.mlp_features(r).cpu().numpy().astype(np.float64)
        h = {k: v.cpu().numpy() for k, v in r.items()}
    v = h["valid"].astype(bool)
    assert v.all()
    fo = OM.features(h["dist"], h["var"], h["aux"][:, 0], h["grad"], h["aux"][:, 2])
    for k in (0, 2, 3, 4, 5):
        assert np.array_equal(f[:, k], fo[:, k]), k
    for k in (1, 6):
        assert (np.abs(f[:, k] - fo[:, k]) <= 5e-7 * np.abs(fo[:, k]) + 1e-12).all(), k
