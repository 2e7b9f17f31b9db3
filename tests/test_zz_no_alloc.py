"""gpdf_query_distance_noalloc through the C ABI: the allocation-free variant
of gpdf_query_distance (its per-cell lists live in a fixed per-GPU array)
gives bitwise the same outputs as gpdf_query_distance, on two calls in a row,
the second with a smaller input, and rejects what it cannot hold."""
import numpy as np
import pytest
import torch

import paper_2407_09649_amd as P
from paper_2407_09649_amd import scenes as S

from parity import small_params

pytestmark = pytest.mark.gpu


def _outs(m, dev):
    return dict(dist=torch.empty(m, device=dev), grad=torch.empty((m, 3), device=dev),
                var=torch.empty(m, device=dev), valid=torch.empty(m, dtype=torch.uint8, device=dev),
                aux=torch.empty((m, 3), device=dev))


def _equal(a, b):
    for k in ("dist", "grad", "var", "valid", "aux"):
        assert torch.equal(a[k], b[k]), k


def test_noalloc_matches_query_distance(dev):
    scene = S.lidar_scene(7)
    pts = S.lidar_frame(scene, (0.0, 0.0, 1.5), np.random.default_rng(7), n_beams=16, n_azimuth=256)
    q = S.shuffle_rows(S.lidar_band_queries(pts, radius_cells=4), 3)
    origin = np.array([0.0, 0.0, 1.5], np.float32)
    with P.Context(small_params(voxel_size=0.1), device=dev) as ctx:
        ctx.train(torch.from_numpy(pts).to(dev))
        for m in (len(q), len(q) // 3):           # second call smaller
            qd = torch.from_numpy(q[:m]).to(dev)
            ref = ctx.query(qd, origin=origin)
            out = ctx.query_noalloc(qd, _outs(m, dev), origin=origin)
            torch.cuda.synchronize()
            _equal(out, ref)
            assert out["valid"].sum() > 0.9 * m
        # unsigned, and a call that asks for no gradient or variance
        qd = torch.from_numpy(q[:5000]).to(dev)
        ref = ctx.query(qd, grad=False, var=False, aux=False)
        o = _outs(5000, dev)
        out = ctx.query_noalloc(qd, dict(dist=o["dist"], valid=o["valid"]))
        torch.cuda.synchronize()
        assert torch.equal(out["dist"], ref["dist"]) and torch.equal(out["valid"], ref["valid"])


def test_noalloc_sphere_knn_and_hardmin(dev):
    sc = S.sphere_scene(2)
    for kw in (dict(selection=P.SEL_KNN, knn_q=8), dict(combine=P.COMB_HARDMIN)):
        with P.Context(small_params(**kw), device=dev) as ctx:
            ctx.train(torch.from_numpy(sc.points).to(dev))
            qd = torch.from_numpy(sc.queries).to(dev)
            ref = ctx.query(qd)
            out = ctx.query_noalloc(qd, _outs(len(sc.queries), dev))
            torch.cuda.synchronize()
            _equal(out, ref)


def test_noalloc_rejects_too_many_cells_and_bf16(dev):
    sc = S.sphere_scene(0)
    with P.Context(small_params(), device=dev) as ctx:
        ctx.train(torch.from_numpy(sc.points).to(dev))
        # one query in each of 70,000 distinct 0.4 m cells
        g = np.stack(np.meshgrid(np.arange(50), np.arange(50), np.arange(28), indexing="ij"), -1).reshape(-1, 3)
        q = ((g + 0.5) * 0.4).astype(np.float32)
        with pytest.raises(P.GpdfError) as ei:
            ctx.query_noalloc(torch.from_numpy(q).to(dev), _outs(len(q), dev))
        assert ei.value.status == 4 and "65536" in str(ei.value)
        # the context still answers afterwards
        qd = torch.from_numpy(sc.queries).to(dev)
        ref = ctx.query(qd)
        out = ctx.query_noalloc(qd, _outs(len(sc.queries), dev))
        torch.cuda.synchronize()
        _equal(out, ref)
    with P.Context(small_params(precision=P.PREC_BF16), device=dev) as ctx:
        ctx.train(torch.from_numpy(sc.points).to(dev))
        with pytest.raises(P.GpdfError) as ei:
            ctx.query_noalloc(torch.from_numpy(sc.queries).to(dev), _outs(len(sc.queries), dev))
        assert ei.value.status == 1
