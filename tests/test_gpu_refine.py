"""The FP64 re-evaluation of the FP32 path's refined queries (those whose
error estimate exceeds the tolerance), against the oracle.

The cluster-major pass takes the (refined query, cluster) pairs of clusters
of at most 256 points; the FP64 query kernel takes every refined query
instead when a model has a larger cluster or a call's pairs exceed the
pass's buffers.  Each route is checked against the oracle at the parity
tolerances, and the two routes against each other.
"""
import numpy as np
import pytest

import oracle as O
import paper_2407_09649_amd as P
from paper_2407_09649_amd import scenes as S

from parity import compare, gpu_query, oracle_params, small_params

pytestmark = pytest.mark.gpu


def _near_queries(ps, n_per, seed):
    """Queries within a few millimetres of the training points: the
    variance 1 - |W k|^2 cancels there, so FP32 refines most of them."""
    rng = np.random.default_rng(seed)
    idx = rng.choice(len(ps.points), n_per * len(ps.sizes), replace=False)
    return (ps.points[idx] + rng.normal(0.0, 0.003, size=(len(idx), 3))).astype(np.float32)


def _run(dev, pts, q, **kw):
    with P.Context(small_params(**kw), device=dev) as ctx:
        import torch
        ctx.train(torch.from_numpy(pts).to(dev))
        g = gpu_query(ctx, q)
        st = ctx.stats()
        params = ctx.params
    return g, st, params


def test_cluster_major_pass_takes_the_pairs(dev):
    ps = S.planar_patches(seed=11, n_patches=96, n_lo=8, n_hi=256, q_per=16)
    q = np.concatenate([ps.queries, _near_queries(ps, 16, 1)])
    g, st, prm = _run(dev, ps.points, q, cluster_size=0.8, max_factor_elems=1 << 25)
    print("refined", st["refined_queries"], "pairs", st["refine_pairs_small"], st["refine_pairs_large"],
          "items", st["refine_items_large"], flush=True)
    assert st["refined_queries"] > 500
    assert st["refine_pairs_small"] > 0 and st["refine_pairs_large"] > 0 and st["refine_items_large"] > 0
    # a refined query pairs with each of its cell's (at most 27) clusters;
    # here each cell's list holds only its own patch
    assert st["refine_pairs_small"] + st["refine_pairs_large"] == st["refined_queries"]
    assert st["refine_items_large"] * 16 >= st["refine_pairs_large"]
    compare(g, O.Model(oracle_params(prm), ps.points).query(q), label="cluster-major")


def test_cluster_above_256_points_takes_the_fp64_kernel(dev):
    ps = S.planar_patches(seed=12, n_patches=24, n_lo=257, n_hi=320, q_per=16)
    q = np.concatenate([ps.queries, _near_queries(ps, 16, 2)])
    g, st, prm = _run(dev, ps.points, q, cluster_size=0.8, max_factor_elems=1 << 25)
    assert st["refined_queries"] > 100
    assert st["refine_pairs_small"] == 0 and st["refine_pairs_large"] == 0
    compare(g, O.Model(oracle_params(prm), ps.points).query(q), label="above 256 points")


def test_too_many_refined_queries_take_the_fp64_kernel(dev):
    # with at most 65,536 queries the pass's result layout holds 2,427
    # refined queries (27 list slots each in 65,536 records); this call
    # refines more, so the FP64 query kernel takes them, and a context with
    # room takes the same call through the pass
    ps = S.planar_patches(seed=13, n_patches=192, n_lo=8, n_hi=200, q_per=4)
    q = np.concatenate([ps.queries, _near_queries(ps, 24, 3)])
    assert len(q) <= 1 << 16
    g_small, st_small, prm = _run(dev, ps.points, q, cluster_size=0.8, max_factor_elems=1 << 25,
                                  max_queries=1 << 16)
    g_big, st_big, _ = _run(dev, ps.points, q, cluster_size=0.8, max_factor_elems=1 << 25,
                            max_queries=1 << 20)
    print("refined", st_small["refined_queries"], "pairs through the pass", st_big["refine_pairs_small"],
          st_big["refine_pairs_large"], flush=True)
    assert st_small["refined_queries"] > 2427
    assert st_small["refine_pairs_small"] == 0 and st_small["refine_pairs_large"] == 0
    assert st_big["refine_pairs_small"] + st_big["refine_pairs_large"] == st_big["refined_queries"]
    ref = O.Model(oracle_params(prm), ps.points).query(q)
    compare(g_small, ref, label="FP64 kernel")
    compare(g_big, ref, label="cluster-major")
    # both routes are FP64 up to the output rounding
    v = g_small["valid"].astype(bool)
    assert np.array_equal(v, g_big["valid"].astype(bool))
    assert np.abs(g_small["dist"][v] - g_big["dist"][v]).max() <= 1e-6
    assert np.abs(g_small["grad"][v] - g_big["grad"][v]).max() <= 1e-5
    assert np.abs(g_small["var"][v] / g_big["var"][v] - 1).max() <= 1e-5
