"""GPU parity of the global GP distance field (G-GPDF, Sec. IV-D): the zero
crossings of the fused grid bit for bit against the oracle's, and the field of
per-leaf GPs trained on them (Q nearest nodes, smooth minimum of Eq. (10))
against the oracle on the same points."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2407_09649_amd as P
from paper_2407_09649_amd import scenes as S

from parity import compare, gpu_query, oracle_params, small_params

pytestmark = pytest.mark.gpu


def _fused(dev, seed, n_frames, beams=16, az=256):
    path = S.sensor_path(seed, n_frames=n_frames)
    scene = S.lidar_scene(seed, keep_clear_xy=path[:, :2], clearance=1.5)
    rng = np.random.default_rng(seed)
    ctx = P.Context(small_params(voxel_size=0.1), device=dev)
    for o in path:
        pts = S.lidar_frame(scene, o, rng, n_beams=beams, n_azimuth=az)
        ctx.fuse(torch.from_numpy(pts).to(dev), np.asarray(o, np.float32))
    torch.cuda.synchronize()
    return ctx


def _oracle_map(g):
    m = O.Map()
    m.merge(g["key"], g["D"].astype(np.float64), g["V"].astype(np.float64), np.ones(len(g["key"])), 0)
    return m


def test_zero_crossings_bitwise(dev):
    ctx = _fused(dev, 4, 3)
    zc = ctx.zero_crossings().cpu().numpy()
    zo = _oracle_map(ctx.export_global()).zero_crossings(0.05)
    assert len(zc) > 10000
    assert zc.shape == zo.shape
    assert np.array_equal(zc.view(np.uint32), zo.view(np.uint32))
    ctx.close()


def test_zero_crossings_empty_grid(dev):
    with P.Context(small_params(), device=dev) as ctx:
        assert ctx.zero_crossings().shape == (0, 3)


def _leaf_params(**kw):
    # one GP per leaf of the grid (8 x 0.05 m), the Q = 8 nearest nodes
    return small_params(cluster_size=0.4, selection=P.SEL_KNN, knn_q=8, max_cluster_points=1024,
                        max_factor_elems=1 << 27, **kw)


def test_ggpdf_parity(dev):
    ctx = _fused(dev, 5, 2)
    zc = ctx.zero_crossings()
    g = ctx.export_global()
    ctx.close()
    pts = zc.cpu().numpy()
    rng = np.random.default_rng(0)
    keys = g["key"][rng.choice(len(g["key"]), 20000)]
    c = np.stack([(keys >> np.uint64(42)) & np.uint64(0x1FFFFF), (keys >> np.uint64(21)) & np.uint64(0x1FFFFF),
                  keys & np.uint64(0x1FFFFF)], 1).astype(np.int64) - (1 << 20)
    q = ((c + 0.5 + rng.uniform(-0.5, 0.5, size=c.shape)) * 0.05).astype(np.float32)
    with P.Context(_leaf_params(), device=dev) as gp:
        gp.train(zc)
        sizes = np.diff(gp.export_model()["off"])
        print(f"G-GPDF: {len(pts)} zero crossings, {len(sizes)} leaves, n median {np.median(sizes):.0f} "
              f"max {sizes.max()}")
        r = gpu_query(gp, q)
        om = O.Model(oracle_params(gp.params), pts)
    res = compare(r, om.query(q), label="G-GPDF")
    assert res["n"] == len(q)
    # near the surface the field is a distance: small where D is small
    near = np.abs(g["D"][np.searchsorted(g["key"], keys)]) < 0.05
    assert np.median(r["dist"][near]) < 0.1


def _lidar_small(seed=7):
    scene = S.lidar_scene(seed)
    return S.lidar_frame(scene, (0.0, 0.0, 1.5), np.random.default_rng(seed), n_beams=16, n_azimuth=256)


@pytest.mark.parametrize("sel", ["knn", "n27"])
def test_lazy_training_matches_eager(dev, sel):
    """A lazily trained model (clusters factored when a query selects them)
    answers bitwise as the eagerly trained one, and factors only what its
    queries select; a second call in another region trains more."""
    if sel == "knn":
        pts = S.sphere_scene(11).points
        kw = dict(selection=P.SEL_KNN, knn_q=8)
        q = S.sphere_eval_queries(12, 4000)
        origin = None
    else:
        pts = _lidar_small()
        kw = dict(voxel_size=0.1)
        q = S.lidar_band_queries(pts, radius_cells=3)
        origin = np.array([0.0, 0.0, 1.5], np.float32)
    # two regions of the query set: one side first, the rest after
    x = q[:, 0]
    cut = np.quantile(x, 0.8)
    first, second = q[x > cut][:3000], q[x <= cut][:3000]
    with P.Context(small_params(**kw), device=dev) as eager, \
            P.Context(small_params(lazy_train=1, **kw), device=dev) as lazy:
        xt = torch.from_numpy(pts).to(dev)
        eager.train(xt)
        lazy.train(xt)
        total = eager.stats()["trained_clusters"]
        assert lazy.stats()["trained_clusters"] == 0
        trained = []
        for part in (first, second):
            a = gpu_query(eager, part, origin)
            b = gpu_query(lazy, part, origin)
            for k in a:
                assert np.array_equal(a[k], b[k], equal_nan=True), (sel, k)
            trained.append(lazy.stats()["trained_clusters"])
        print(f"lazy {sel}: trained {trained} of {total}")
        assert 0 < trained[0] < total and trained[0] <= trained[1] <= total, (trained, total)
        gpu_query(lazy, first, origin)              # nothing new to train
        assert lazy.stats()["trained_clusters"] == trained[1]


def test_ggpdf_lazy_knn_parity(dev):
    """The G-GPDF as the paper queries it: only the Q nearest nodes of the
    queries are trained (lazily), against the oracle's fully trained field."""
    ctx = _fused(dev, 6, 2)
    zc = ctx.zero_crossings()
    g = ctx.export_global()
    ctx.close()
    rng = np.random.default_rng(3)
    keys = g["key"][rng.choice(len(g["key"]), 5000)]
    c = np.stack([(keys >> np.uint64(42)) & np.uint64(0x1FFFFF), (keys >> np.uint64(21)) & np.uint64(0x1FFFFF),
                  keys & np.uint64(0x1FFFFF)], 1).astype(np.int64) - (1 << 20)
    q = ((c + 0.5 + rng.uniform(-0.5, 0.5, size=c.shape)) * 0.05).astype(np.float32)
    q = q[q[:, 0] > np.quantile(q[:, 0], 0.7)]      # one side of the map
    with P.Context(_leaf_params(lazy_train=1), device=dev) as gp:
        gp.train(zc)
        r = gpu_query(gp, q)
        st = gp.stats()
        om = O.Model(oracle_params(gp.params), zc.cpu().numpy())
    print(f"lazy G-GPDF: trained {st['trained_clusters']} of {st['clusters']} leaves for {len(q)} queries")
    assert st["trained_clusters"] < st["clusters"]
    compare(r, om.query(q), label="lazy G-GPDF")
