"""The FP64 trainers at the bounds of their size buckets, against the oracle.

Clusters of 65-256 points go to the blocked trainer, in four buckets by
16-row tile rows T: T <= 6, T <= 8 and T <= 12 with the tiles in LDS, and
T <= 16 with the tiles in the FP64 workspace; smaller clusters to the lane
and wavefront trainers.  Every cluster here is one planar patch alone in its
cell, of an exact size at a bucket bound, so each trainer instance meets
both ends of its range.  Exact duplicate points without a noise term make a
cluster's K singular, the case where the factorisation must stop and mark
the cluster (Eq. (1); a pivot at or below 1e-10 (1 + s^2)).
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2407_09649_amd as P

from parity import compare, export_equal, gpu_query, oracle_params, small_params

pytestmark = pytest.mark.gpu

CELL = 0.8


def _patches(sizes, seed, q_per=48, dup_from=None):
    """One planar patch of sizes[i] points in cell (2i, 0, 0) (patches two
    cells apart), q_per queries uniform in each patch's cell.  Patches of at
    least dup_from points have one point repeat another exactly."""
    rng = np.random.default_rng(seed)
    pts, qs = [], []
    for i, n in enumerate(sizes):
        lo = np.array([2.0 * i, 0.0, 0.0]) * CELL
        c = lo + 0.5 * CELL
        nrm = rng.normal(size=3)
        nrm /= np.linalg.norm(nrm)
        e1 = np.cross(nrm, [1.0, 0.0, 0.0] if abs(nrm[0]) < 0.9 else [0.0, 1.0, 0.0])
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(nrm, e1)
        uv = rng.uniform(-0.2, 0.2, size=(n, 2))
        h = rng.normal(0.0, 0.01, size=n)
        p = (c + uv[:, :1] * e1 + uv[:, 1:] * e2 + h[:, None] * nrm).astype(np.float32)
        if dup_from is not None and n >= dup_from:
            p[n // 2] = p[3]
        pts.append(p)
        qs.append(lo + rng.uniform(0.0, CELL, size=(q_per, 3)))
    return np.concatenate(pts), np.concatenate(qs).astype(np.float32)


def _run(dev, pts, q, **kw):
    with P.Context(small_params(cluster_size=CELL, max_factor_elems=1 << 25, **kw), device=dev) as ctx:
        ctx.train(torch.from_numpy(pts).to(dev))
        om = O.Model(oracle_params(ctx.params), pts)
        e = export_equal(ctx, om, alpha_rtol=1e-8)
        g = gpu_query(ctx, q)
        st = ctx.stats()
    return e, g, st, om


@pytest.mark.parametrize("kw", [{}, dict(kernel=P.KERNEL_SE, length_scale=0.15)], ids=["matern32", "se"])
def test_bucket_bounds_against_the_oracle(dev, kw):
    # lane and wavefront trainers (8, 9, 64), then the blocked trainer's four
    # buckets at both ends: 65-96, 97-128, 129-192, 193-256 points; with the
    # noise term K + s^2 I stays conditioned well enough for alpha to agree
    # within 1e-8 relative under either kernel
    sizes = [8, 9, 64, 65, 96, 97, 128, 129, 192, 193, 256]
    pts, q = _patches(sizes, seed=21)
    e, g, st, om = _run(dev, pts, q, **kw)
    print("cluster sizes", np.diff(e["off"]).tolist(), flush=True)
    assert sorted(np.diff(e["off"]).tolist()) == sorted(sizes)
    assert e["pd"].all() and st["nonpd_clusters"] == 0
    compare(g, om.query(q), label="bucket bounds")


def test_singular_clusters_of_every_blocked_bucket_are_excluded(dev):
    # one exact duplicate in each blocked-trainer cluster and no noise term:
    # each K is singular and the factorisation stops at a pivot of rounding
    # size; the clusters of 4 distinct points stay positive definite
    sizes = [4, 80, 4, 120, 4, 180, 4, 230]
    pts, q = _patches(sizes, seed=22, dup_from=65)
    e, g, st, om = _run(dev, pts, q, noise_sigma=0.0)
    sz = np.diff(e["off"])
    assert om.nonpd == 4 and st["nonpd_clusters"] == 4
    assert not e["pd"][sz > 64].any() and e["pd"][sz <= 8].all()
    assert st["status_bits"] & 8
    compare(g, om.query(q), label="singular blocked clusters")
