"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Sizes are those the oracle finishes in seconds while spanning many
wavefront chunks, cells of every size class (n <= 16, 32, 64 and the
64-row panel path) and ragged tails; the full-size LiDAR frame is checked on
a sample of its queries in the launch configuration the benchmark times.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2407_09649_amd as P
from paper_2407_09649_amd import scenes as S

from parity import compare, export_equal, gpu_query, oracle_params, signed_dist_err, small_params

pytestmark = pytest.mark.gpu


def _ctx(dev, **kw):
    return P.Context(small_params(**kw), device=dev)


def _train(ctx, pts):
    ctx.train(torch.from_numpy(np.ascontiguousarray(pts, np.float32)).to(ctx.device))


# ---------------------------------------------------------------------------
# sphere scenes (2,048 raw points, 0.4 m cells, 10,000 queries)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_sphere_fp32_parity(dev, seed):
    sc = S.sphere_scene(seed)
    with _ctx(dev) as ctx:
        _train(ctx, sc.points)
        om = O.Model(oracle_params(ctx.params), sc.points)
        export_equal(ctx, om)
        g = gpu_query(ctx, sc.queries)
        st = ctx.stats()
    r = compare(g, om.query(sc.queries), label=f"sphere seed {seed}")
    assert r["n"] == st["valid_queries"] > 3000
    assert st["refined_queries"] < 0.05 * st["valid_queries"]


def test_sphere_fp64_mode_parity(dev):
    sc = S.sphere_scene(0)
    with _ctx(dev, precision=P.PREC_FP64) as ctx:
        _train(ctx, sc.points)
        g = gpu_query(ctx, sc.queries)
    compare(g, O.Model(oracle_params(ctx.params), sc.points).query(sc.queries), fp64=True,
            label="fp64")


@pytest.mark.parametrize("mode", ["se", "hardmin", "paper_mean"])
def test_sphere_modes_parity(dev, mode):
    kw = dict(se=dict(kernel=P.KERNEL_SE), hardmin=dict(combine=P.COMB_HARDMIN),
              paper_mean=dict(grad_mode=P.GRAD_PAPER_MEAN))[mode]
    sc = S.sphere_scene(3)
    with _ctx(dev, **kw) as ctx:
        _train(ctx, sc.points)
        g = gpu_query(ctx, sc.queries)
        om = O.Model(oracle_params(ctx.params), sc.points)
    compare(g, om.query(sc.queries), label=mode, closest_node=(mode == "hardmin"))


def test_lidar_closest_node_parity(dev):
    """The closest-node rule on a signed LiDAR scan: where two leaves give
    nearly the same distance the FP32 argmin may take the other one, and the
    result must then be that node's (the oracle's second answer)."""
    pts = _lidar(7, beams=16, az=256)
    q = S.lidar_band_queries(pts, radius_cells=4)
    origin = np.array([0.0, 0.0, 1.5], np.float32)
    with _ctx(dev, voxel_size=0.1, combine=P.COMB_HARDMIN) as ctx:
        _train(ctx, pts)
        g = gpu_query(ctx, q, origin=origin)
        om = O.Model(oracle_params(ctx.params), pts)
    o = om.query(q, origin=origin)
    r = compare(g, o, label="lidar hardmin", closest_node=True)
    assert r["node_alt"] <= 0.01 * r["n"]


def test_knn_far_field_parity(dev):
    sc = S.sphere_scene(10000)
    q = S.sphere_eval_queries(20000, 30000)
    with _ctx(dev, selection=P.SEL_KNN, knn_q=8) as ctx:
        _train(ctx, sc.points)
        g = gpu_query(ctx, q)
        om = O.Model(oracle_params(ctx.params), sc.points)
    r = compare(g, om.query(q), label="knn")
    assert r["n"] == len(q)


# ---------------------------------------------------------------------------
# LiDAR frames: voxel downsampling, 8^3-voxel leaves, signed queries
# ---------------------------------------------------------------------------
def _lidar(seed, beams=64, az=1024):
    sc = S.lidar_scene(seed)
    rng = np.random.default_rng(seed)
    pts = S.lidar_frame(sc, (0.0, 0.0, 1.5), rng, n_beams=beams, n_azimuth=az)
    return pts


def test_small_lidar_frame_full_parity(dev):
    pts = _lidar(7, beams=16, az=256)
    q = S.lidar_band_queries(pts, radius_cells=4)
    q = S.shuffle_rows(q, 1)
    origin = np.array([0.0, 0.0, 1.5], np.float32)
    with _ctx(dev, voxel_size=0.1) as ctx:
        _train(ctx, pts)
        om = O.Model(oracle_params(ctx.params), pts)
        export_equal(ctx, om)
        g = gpu_query(ctx, q, origin=origin)
    r = compare(g, om.query(q, origin=origin), label="small lidar")
    assert r["n"] > 100000
    assert (g["dist"][g["valid"].astype(bool)] < 0).any()  # both sides of surfaces


def test_unrequested_outputs_are_not_refined(dev):
    """The FP64 re-evaluation serves the outputs a call asks for: without a
    gradient buffer no query is redone for its gradient, without a variance
    buffer none for its variance, and the requested outputs keep their
    tolerance against the oracle."""
    pts = _lidar(7, beams=16, az=256)
    q = S.lidar_band_queries(pts, radius_cells=4)
    origin = np.array([0.0, 0.0, 1.5], np.float32)
    with _ctx(dev, voxel_size=0.1) as ctx:
        _train(ctx, pts)
        qd = torch.from_numpy(q).to(dev)
        full = ctx.query(qd, origin=origin)
        st_full = ctx.stats()
        dv = ctx.query(qd, origin=origin, grad=False, aux=False)
        st_dv = ctx.stats()
        d = ctx.query(qd, origin=origin, grad=False, var=False, aux=False)
        st_d = ctx.stats()
        om = O.Model(oracle_params(ctx.params), pts)
    assert st_full["refine_grad"] > 0 and st_full["refine_var"] > 0
    assert st_dv["refine_grad"] == 0 and st_d["refine_grad"] == 0 and st_d["refine_var"] == 0
    assert st_d["refined_queries"] <= st_dv["refined_queries"] < st_full["refined_queries"]
    ref = om.query(q, origin=origin)
    v = ref["valid"]
    for out in (full, dv, d):
        assert np.array_equal(out["valid"].cpu().numpy().astype(bool), v)
        assert signed_dist_err(out["dist"].cpu().numpy(), ref).max() <= 1e-4
    assert np.abs(dv["var"].cpu().numpy()[v] / ref["var"][v] - 1).max() <= 2e-3


def test_full_lidar_frame_sampled_parity(dev):
    """The benchmark's workload: one 64 x 1024 scan, ~4.9M band queries,
    evaluated in one call; 30,000 sampled queries against the oracle."""
    pts = _lidar(1)
    q = S.lidar_band_queries(pts)
    origin = np.array([0.0, 0.0, 1.5], np.float32)
    with P.Context(P.Params.default(voxel_size=0.1), device=dev) as ctx:
        _train(ctx, pts)
        om = O.Model(oracle_params(ctx.params), pts)
        export_equal(ctx, om)
        g = gpu_query(ctx, q, origin=origin)
        st = ctx.stats()
    assert st["queries"] == len(q) and st["valid_queries"] > 0.99 * len(q)
    assert st["refined_queries"] < 0.02 * len(q)
    idx = np.random.default_rng(0).choice(len(q), 30000, replace=False)
    gs = {k: v[idx] for k, v in g.items()}
    compare(gs, om.query(q[idx], origin=origin), label="full lidar sample")
    # every query is decided: valid ones are finite, invalid ones +inf
    v = g["valid"].astype(bool)
    assert np.isfinite(g["dist"][v]).all() and np.isinf(g["dist"][~v]).all()


# ---------------------------------------------------------------------------
# uneven planar patches: n from 8 to 256 (all size classes and panels)
# ---------------------------------------------------------------------------
def test_planar_patches_parity(dev):
    ps = S.planar_patches(seed=3, n_patches=384, q_per=32)
    with _ctx(dev, cluster_size=0.8, max_factor_elems=1 << 25) as ctx:
        _train(ctx, ps.points)
        om = O.Model(oracle_params(ctx.params), ps.points)
        e = export_equal(ctx, om, alpha_rtol=1e-8)
        g = gpu_query(ctx, ps.queries)
    sizes = np.diff(e["off"])
    assert sizes.min() <= 16 and sizes.max() > 192
    compare(g, om.query(ps.queries), label="patches")


# ---------------------------------------------------------------------------
# edge cases and failure handling
# ---------------------------------------------------------------------------
def test_empty_inputs(dev):
    sc = S.sphere_scene(0, n_points=64, n_queries=16)
    with _ctx(dev) as ctx:
        with pytest.raises(P.GpdfError) as ei:
            ctx.query(torch.from_numpy(sc.queries).to(dev))
        assert ei.value.status == 5  # not trained
        _train(ctx, sc.points[:0])
        g = gpu_query(ctx, sc.queries)
        assert not g["valid"].any() and np.isinf(g["dist"]).all()
        _train(ctx, sc.points)
        g0 = gpu_query(ctx, sc.queries[:0])
        assert g0["dist"].shape == (0,)


def test_nonfinite_inputs_are_skipped_and_counted(dev):
    sc = S.sphere_scene(4, n_points=600, n_queries=500)
    pts = sc.points.copy()
    pts[[3, 77, 500], [0, 1, 2]] = [np.nan, np.inf, -np.inf]
    q = sc.queries.copy()
    q[[5, 6], [2, 0]] = [np.nan, np.inf]
    with _ctx(dev) as ctx:
        _train(ctx, pts)
        g = gpu_query(ctx, q)
        st = ctx.stats()
        om = O.Model(oracle_params(ctx.params), pts)
    assert st["skipped_points"] == 3 and om.skipped == 3
    assert st["status_bits"] & 4
    assert not g["valid"][5] and not g["valid"][6]
    compare(g, om.query(q), label="nonfinite")


def test_non_positive_definite_cluster_is_excluded(dev):
    # three identical points and no noise term: K is singular
    pts = np.array([[0.1, 0.1, 0.1]] * 3 + [[0.15, 0.1, 0.1], [1.1, 0.1, 0.1]], np.float32)
    q = np.array([[0.1, 0.1, 0.2], [1.1, 0.1, 0.2], [0.5, 0.1, 0.1]], np.float32)
    with _ctx(dev, noise_sigma=0.0) as ctx:
        _train(ctx, pts)
        st = ctx.stats()
        g = gpu_query(ctx, q)
        om = O.Model(oracle_params(ctx.params), pts)
    assert st["nonpd_clusters"] == om.nonpd == 1
    assert st["status_bits"] & 8
    compare(g, om.query(q), label="nonpd")


def test_capacity_errors(dev):
    sc = S.sphere_scene(0, n_points=300)
    with P.Context(small_params(max_points=256, max_queries=128), device=dev) as ctx:
        with pytest.raises(P.GpdfError) as ei:
            _train(ctx, sc.points)
        assert ei.value.status == 4
        _train(ctx, sc.points[:200])
        with pytest.raises(P.GpdfError) as ei:
            ctx.query(torch.from_numpy(sc.queries[:200]).to(dev))
        assert ei.value.status == 4
    big = np.random.default_rng(0).uniform(0.01, 0.39, size=(300, 3)).astype(np.float32)
    with P.Context(small_params(max_cluster_points=256), device=dev) as ctx:
        with pytest.raises(P.GpdfError) as ei:
            _train(ctx, big)  # one 0.4 m cell with 300 points
        assert ei.value.status == 4


def test_results_are_deterministic_and_order_independent(dev):
    pts = _lidar(9, beams=16, az=256)
    q = S.lidar_band_queries(pts, radius_cells=3)
    perm = np.random.default_rng(2).permutation(len(q))
    origin = np.array([0.0, 0.0, 1.5], np.float32)
    with _ctx(dev, voxel_size=0.1) as ctx:
        _train(ctx, pts)
        a = gpu_query(ctx, q, origin=origin)
        b = gpu_query(ctx, q, origin=origin)
        c = gpu_query(ctx, q[perm], origin=origin)
        _train(ctx, pts[np.random.default_rng(3).permutation(len(pts))])
        d = gpu_query(ctx, q, origin=origin)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k][perm], c[k]), k
        # voxel mode fixes the member order, so training order does not matter
        assert np.array_equal(a[k], d[k]), k


def test_nearest_distance_brute_force(dev):
    rng = np.random.default_rng(5)
    p = rng.normal(size=(3000, 3)).astype(np.float32)
    q = rng.normal(size=(5000, 3)).astype(np.float32)
    with _ctx(dev) as ctx:
        d = ctx.nearest_distance(torch.from_numpy(p).to(dev), torch.from_numpy(q).to(dev))
        d = d.cpu().numpy()
    ref = O.nearest_distance(p, q)
    assert np.abs(d - ref).max() <= 1e-6 * max(1.0, ref.max())


def _adversarial_coords(h):
    """FP32 values on and next to cell boundaries: exact multiples of h, their
    FP32 neighbours, signed zeros, tiny values and the ends of the 21-bit key
    range (+-2^20 cells)."""
    lim = np.float32((1 << 20) * h)
    base = [0.0, -0.0, h, -h, 3 * h, -3 * h, 1.0, -1.0, 12.3, -12.3, 1e-30, -1e-30,
            0.2999999, 0.7, float(lim) * 0.5, -float(lim) * 0.5, float(lim), -float(lim),
            float(np.nextafter(lim, np.float32(0))), float(np.nextafter(-lim, np.float32(0)))]
    vals = []
    for b in base:
        f = np.float32(b)
        vals += [f, np.nextafter(f, np.float32(np.inf)), np.nextafter(f, np.float32(-np.inf))]
    vals += [np.float32(k * h) for k in range(-50, 51, 7)]
    return np.array(vals, np.float32)


@pytest.mark.parametrize("mode", ["voxel", "raw"])
def test_adversarial_keys_bitwise(dev, mode):
    """Keys, voxel centres, cluster membership and the per-query cell
    selection on coordinates chosen to break a wrong floor, a wrong rounding
    or a wrong range check: the exported model equals the oracle's bit for
    bit, the same points are skipped, and the queries see the same clusters."""
    kw = dict(voxel_size=0.1) if mode == "voxel" else dict(cluster_size=0.4)
    h = 0.1 if mode == "voxel" else 0.4
    v = _adversarial_coords(h)
    pts = np.stack([v, v[::-1], np.roll(v, 3)], axis=1)
    pts = np.concatenate([pts, pts[:, [1, 2, 0]], pts[:, [2, 0, 1]]]).astype(np.float32)
    q = np.concatenate([pts, pts + np.float32(h / 3)]).astype(np.float32)
    with _ctx(dev, **kw) as ctx:
        _train(ctx, pts)
        st = ctx.stats()
        om = O.Model(oracle_params(ctx.params), pts)
        export_equal(ctx, om)
        g = gpu_query(ctx, q)
    assert st["skipped_points"] == om.skipped > 0
    assert st["points"] == om.npoints and st["clusters"] == om.nclusters
    ref = om.query(q)
    assert np.array_equal(g["valid"].astype(bool), ref["valid"])
    v = ref["valid"]
    assert v.sum() > 0
    assert np.array_equal(g["aux"][v, 2], ref["aux"][v, 2])
