"""Pins of the oracle's surface-property GP and its fusion (Eq. (6); Sec. IV-C).

Each check compares the oracle with something it does not compute itself:
the brute-force mean of the raw properties of a voxel, the identity that a GP
posterior mean at a training input equals c - s^2 (K + s^2 I)^{-1} c, the
linearity of Eq. (6) in c, per-cluster results of separately trained models,
the product of Gaussian observations, the weighted mean of TSDF weights, and
the exact reproduction of an affine field by trilinear interpolation.
"""
import numpy as np
import pytest

import oracle as O

S2 = 0.01 ** 2


def _cloud(seed, n, lo=-0.6, hi=0.6):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(n, 3)).astype(np.float32), rng


def _key3(x, h):
    return [tuple(np.floor(np.float64(v) / h).astype(np.int64)) for v in x]


def test_voxel_property_is_the_input_order_mean():
    # several raw points per voxel: the training point's property is the mean
    # of its raw points' properties, summed in FP64 in input order
    rng = np.random.default_rng(1)
    h = 0.1
    cells = rng.integers(-6, 6, size=(60, 3))
    reps = rng.integers(1, 6, size=60)
    pts = np.concatenate([(c + rng.uniform(0.05, 0.95, size=(r, 3))) * h for c, r in zip(cells, reps)])
    perm = rng.permutation(len(pts))
    pts = pts[perm].astype(np.float32)
    prop = rng.uniform(-2, 2, size=len(pts)).astype(np.float32)
    m = O.Model(O.Params(voxel=h), pts, prop=prop)
    sums, counts = {}, {}
    for k, c in zip(_key3(pts, h), prop):
        sums[k] = sums.get(k, 0.0) + float(c)
        counts[k] = counts.get(k, 0) + 1
    e = m.export()
    got = m.props()["prop"]
    assert len(got) == len(sums) == m.npoints
    for x, g in zip(e["points"], got):
        k = tuple(np.floor(np.float64(x) / h).astype(np.int64))
        assert g == sums[k] / counts[k]          # bitwise


def test_raw_mode_property_is_the_point_property():
    pts, rng = _cloud(2, 300)
    prop = rng.uniform(0, 1, size=300).astype(np.float32)
    m = O.Model(O.Params(cell=0.4), pts, prop=prop)
    e = m.export()
    idx = {tuple(p): i for i, p in enumerate(pts.tolist())}
    src = np.array([idx[tuple(p)] for p in e["points"].tolist()])
    assert np.array_equal(m.props()["prop"], prop[src].astype(np.float64))


def test_beta_solves_the_property_system():
    # (K + s^2 I) beta = c per cluster, and a constant property gives
    # beta = kappa alpha (the occupancy system has right-hand side 1)
    pts, rng = _cloud(3, 400)
    prop = rng.uniform(0, 1, size=400).astype(np.float32)
    prm = O.Params(cell=0.4)
    m = O.Model(prm, pts, prop=prop)
    e, pr = m.export(), m.props()
    for c in range(m.nclusters):
        a, b = e["off"][c], e["off"][c + 1]
        P = e["points"][a:b].astype(np.float64)
        r = np.sqrt(((P[:, None] - P[None]) ** 2).sum(-1)) * np.sqrt(3) / 0.2
        A = (1 + r) * np.exp(-r) + S2 * np.eye(b - a)
        res = A @ pr["beta"][a:b] - pr["prop"][a:b]
        assert np.abs(res).max() <= 1e-9 * (1 + np.abs(A).sum(1).max() * np.abs(pr["beta"][a:b]).max())
    kappa = np.float32(0.625)
    mk = O.Model(prm, pts, prop=np.full(400, kappa, np.float32))
    assert np.abs(mk.props()["beta"] - float(kappa) * e["alpha"]).max() <= 1e-12 * (1 + np.abs(e["alpha"]).max())


def _one_cell_model(seed, n=40, prop=None):
    # every point in the cell [0, 0.4)^3, queries nearby see that cluster only
    rng = np.random.default_rng(seed)
    pts = rng.uniform(0.02, 0.38, size=(n, 3)).astype(np.float32)
    c = rng.uniform(0, 1, size=n).astype(np.float32) if prop is None else prop
    return O.Model(O.Params(cell=0.4), pts, prop=c), pts, c, rng


def test_property_posterior_at_the_training_points():
    # the GP posterior mean at a training input is K beta = c - s^2 beta, and
    # the property variance is the latent variance of Eq. (2) (same kernel,
    # same noise)
    m, pts, c, _ = _one_cell_model(4)
    assert m.nclusters == 1
    r = m.query(pts)
    pr = m.props()
    e = m.export()
    order = {tuple(p): i for i, p in enumerate(e["points"].tolist())}
    j = np.array([order[tuple(p)] for p in pts.tolist()])
    expect = pr["prop"][j] - S2 * pr["beta"][j]
    assert np.abs(r["prop"] - expect).max() <= 1e-9
    assert np.array_equal(r["prop_var"], r["aux"][:, 1])
    # far from the data the posterior returns to the prior: mean 0, variance 1
    far = np.array([[0.2, 0.2, 0.79]], np.float32)
    rf = m.query(far)
    assert rf["valid"][0] and abs(rf["prop"][0]) < 0.2 and rf["prop_var"][0] > 0.5


def test_property_is_linear_in_c_and_scales_the_occupancy():
    pts, rng = _cloud(5, 500)
    q = rng.uniform(-0.7, 0.7, size=(300, 3)).astype(np.float32)
    prm = O.Params(cell=0.4)
    c1 = rng.uniform(0, 1, size=500).astype(np.float32)
    c2 = rng.uniform(-1, 1, size=500).astype(np.float32)
    # c1 + c2 rounded to FP32 is the input of the third model; use values whose
    # FP32 sum is exact (multiples of 2^-10 below 2)
    c1 = np.round(c1 * 1024) / 1024
    c2 = np.round(c2 * 1024) / 1024
    r1 = O.Model(prm, pts, prop=c1).query(q)
    r2 = O.Model(prm, pts, prop=c2).query(q)
    r12 = O.Model(prm, pts, prop=(c1 + c2).astype(np.float32)).query(q)
    v = r1["valid"]
    assert v.sum() > 100
    assert np.abs(r12["prop"][v] - r1["prop"][v] - r2["prop"][v]).max() <= 1e-9
    # the weights do not depend on c
    assert np.array_equal(r1["prop_var"], r2["prop_var"])
    # c = 1 reproduces the latent occupancy on a one-cluster model
    m1, pts1, _, rng1 = _one_cell_model(6, prop=np.ones(40, np.float32))
    q1 = rng1.uniform(0.0, 0.4, size=(200, 3)).astype(np.float32)
    r = m1.query(q1)
    assert np.abs(r["prop"] - r["aux"][:, 0]).max() <= 1e-12


def test_property_combination_against_separately_trained_clusters():
    # KNN with Q >= clusters selects all of them: the property and its
    # variance are the distance's smooth-minimum weights applied to the
    # per-cluster property and latent variance; under the closest-node rule,
    # those of the closest node
    pts, rng = _cloud(7, 240, -0.8, 0.8)
    prop = rng.uniform(0, 1, size=240).astype(np.float32)
    prm = O.Params(selection=1, knn_q=64, cell=0.8)
    q = rng.uniform(-1.0, 1.0, size=(60, 3)).astype(np.float32)
    m = O.Model(prm, pts, prop=prop)
    e = m.export()
    assert 1 < m.nclusters <= 64
    idx = {tuple(p): i for i, p in enumerate(pts.tolist())}
    res = []
    for c in range(m.nclusters):
        sub = e["points"][e["off"][c]:e["off"][c + 1]]
        cs = prop[[idx[tuple(p)] for p in sub.tolist()]]
        res.append(O.Model(prm.copy(cell=1e4, selection=0), sub, prop=cs).query(q))
    D = np.stack([x["dist"] for x in res], 1)
    Cq = np.stack([x["prop"] for x in res], 1)
    U = np.stack([x["aux"][:, 1] for x in res], 1)
    w = np.exp(-100 * (D - D.min(1, keepdims=True)))
    r = m.query(q)
    assert np.abs(r["prop"] - (w * Cq).sum(1) / w.sum(1)).max() <= 1e-12
    assert np.abs(r["prop_var"] - (w * U).sum(1) / w.sum(1)).max() <= 1e-12
    amin = D.argmin(1)
    ii = np.arange(len(q))
    rh = O.Model(prm.copy(combine=1), pts, prop=prop).query(q)
    assert np.abs(rh["prop"] - Cq[ii, amin]).max() <= 1e-12
    assert np.abs(rh["prop_var"] - U[ii, amin]).max() <= 1e-15


def _merge_seq(rule, obs):
    g = O.Map()
    k = np.array([7], np.uint64)
    for f, (c, w) in enumerate(obs):
        g.merge(k, [0.1], [0.01], [1], f, rule=rule, prop=[c], prop_var=[w])
    return g.export()


def test_property_fusion_is_the_product_of_gaussians():
    # Eq. (7)-(8) with the property variance: after any number of
    # observations (c_i, w_i) the voxel holds the precision-weighted mean and
    # the combined variance, whatever the order
    obs = [(0.2, 0.5), (0.9, 0.125), (0.4, 0.3), (0.7, 2.0)]
    c = np.array([o[0] for o in obs])
    w = np.array([o[1] for o in obs])
    C_ref = (c / w).sum() / (1 / w).sum()
    W_ref = 1 / (1 / w).sum()
    for perm in ([0, 1, 2, 3], [3, 1, 0, 2]):
        ex = _merge_seq(0, [obs[i] for i in perm])
        assert abs(ex["C"][0] - C_ref) <= 1e-15 and abs(ex["W"][0] / W_ref - 1) <= 1e-14


def test_property_fusion_tsdf_weights():
    # Eq. (9) with the property variance: weights 1 - w accumulate and C is
    # their weighted mean
    obs = [(0.2, 0.5), (0.9, 0.125), (0.4, 0.3)]
    c = np.array([o[0] for o in obs])
    om = 1 - np.array([o[1] for o in obs])
    ex = _merge_seq(1, obs)
    assert abs(ex["C"][0] - np.average(c, weights=om)) <= 1e-15
    assert abs(ex["W"][0] - om.sum()) <= 1e-15


def test_property_fusion_skips_unusable_observations():
    k = np.array([3, 5], np.uint64)
    g = O.Map()
    # voxel 3 has a usable property, voxel 5 not (variance 0): 5 holds none
    g.merge(k, [0.1, 0.2], [0.01, 0.01], [1, 1], 0, prop=[0.5, 0.6], prop_var=[0.25, 0.0])
    ex = g.export()
    assert ex["C"][0] == 0.5 and ex["W"][0] == 0.25 and np.isnan(ex["C"][1]) and np.isnan(ex["W"][1])
    # unusable observations (NaN, infinite, zero variance) leave voxel 3 alone;
    # voxel 5 takes its first usable one as is
    for i, bad in enumerate((np.nan, np.inf, 0.0)):
        g.merge(k, [0.1, 0.2], [0.01, 0.01], [1, 1], 1 + i, prop=[0.9, 0.8], prop_var=[bad, 0.5])
        ex = g.export()
        assert ex["C"][0] == 0.5 and ex["W"][0] == 0.25
        assert (ex["C"][1] == 0.8) if i == 0 else abs(ex["C"][1] - 0.8) <= 1e-15
    # a voxel skipped for its distance skips its property too
    g.merge(k, [0.1, 0.2], [0.01, 0.01], [0, 1], 2, prop=[0.0, 0.8], prop_var=[0.25, 0.5])
    assert g.export()["C"][0] == 0.5
    # TSDF: a weight 1 - w <= 0 is unusable
    g2 = O.Map()
    g2.merge(k[:1], [0.1], [0.01], [1], 0, rule=1, prop=[0.3], prop_var=[1.0])
    assert np.isnan(g2.export()["C"][0])


def test_global_property_query_reproduces_an_affine_field():
    h = 0.05
    cc = np.stack(np.meshgrid(*[np.arange(-3, 4)] * 3, indexing="ij"), -1).reshape(-1, 3)
    key = (((cc[:, 0] + (1 << 20)).astype(np.uint64) << np.uint64(42)) |
           ((cc[:, 1] + (1 << 20)).astype(np.uint64) << np.uint64(21)) |
           (cc[:, 2] + (1 << 20)).astype(np.uint64))
    o = np.argsort(key)
    key, cc = key[o], cc[o]
    centre = (cc + 0.5) * h
    a, b = np.array([0.7, -1.1, 0.4]), 0.3
    g = O.Map()
    n = len(key)
    g.merge(key, np.full(n, 0.1), np.full(n, 0.01), np.ones(n, np.uint8), 0,
            prop=centre @ a + b, prop_var=np.full(n, 0.01))
    rng = np.random.default_rng(9)
    q = rng.uniform(-2.5 * h, 3.5 * h, size=(500, 3)).astype(np.float32)
    r = g.query_prop(h, q)
    assert r["valid"].all()
    assert np.abs(r["prop"] - (q.astype(np.float64) @ a + b)).max() <= 1e-12
    # outside the block, or next to a voxel with no property: invalid
    assert not g.query_prop(h, np.array([[0.2, 0.0, 0.0]], np.float32))["valid"][0]
    g.merge(key[:1], [0.1], [0.01], [1], 1, prop=[np.nan], prop_var=[0.01])
    assert not np.isnan(g.export()["C"][0])    # an unusable observation does not erase it


def test_fusion_with_properties_takes_the_query_results():
    # first frame: every fused voxel holds the property query at its centre
    pts, rng = _cloud(10, 400)
    prop = rng.uniform(0, 1, size=400).astype(np.float32)
    prm = O.Params(voxel=0.1, fuse_voxel=0.05, fuse_band=0.1)
    m = O.Model(prm, pts, prop=prop)
    g = O.Map()
    origin = np.array([0.0, 0.0, 3.0], np.float32)
    n, sk = g.fuse(m, origin, 0)
    ex = g.export()
    x = O.voxel_centres(ex["key"], 0.05)
    r = m.query(x, origin)
    assert np.array_equal(ex["C"], r["prop"]) and np.array_equal(ex["W"], r["prop_var"])
